"""The im2col layout (section 3.2, appendix A.4: the windows of the image
scanned into one vector, slot k*windows + w for kernel offset k = ky*K + kx
and window w = oy*OW + ox) pinned against a direct sliding-window
convolution, for the oracle's and the library's host im2col, on non-square
images with non-symmetric kernels: the product of the kernel with the im2col
matrix must be the convolution itself.  Planted transpositions (of the
kernel offset, of the window index) must fail the same check."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.plain_ref import conv2d_direct, cnn_fp64

SHAPES = [(28, 28, 7, 3), (10, 13, 3, 2), (11, 9, 4, 1), (9, 16, 5, 4)]


def conv_via_im2col(vec, kernel, h, w, k, stride):
    oh, ow = (h - k) // stride + 1, (w - k) // stride + 1
    return (kernel.reshape(k * k) @ vec.reshape(k * k, oh * ow)).reshape(oh, ow)


def im2col_plain(img, k, stride, swap_offset=False, swap_window=False):
    """A Python im2col with optional planted mistakes (test of the pin)."""
    h, w = img.shape
    oh, ow = (h - k) // stride + 1, (w - k) // stride + 1
    out = np.zeros((k * k, oh * ow))
    for ky in range(k):
        for kx in range(k):
            for oy in range(oh):
                for ox in range(ow):
                    ko = kx * k + ky if swap_offset else ky * k + kx
                    wi = ox * oh + oy if swap_window else oy * ow + ox
                    out[ko, wi] = img[oy * stride + ky, ox * stride + kx]
    return out.reshape(-1)


@pytest.mark.parametrize("h,w,k,stride", SHAPES)
def test_oracle_im2col_is_the_convolution(h, w, k, stride):
    rng = np.random.default_rng(h * 100 + w)
    img = rng.uniform(0, 1, (h, w))
    kern = rng.normal(0, 1, (k, k))
    want = conv2d_direct(img, kern, stride)
    got = conv_via_im2col(O.im2col(img, k, stride), kern, h, w, k, stride)
    assert np.abs(got - want).max() < 1e-12
    # the planted Python copy agrees exactly with the oracle when unplanted
    assert np.array_equal(im2col_plain(img, k, stride), O.im2col(img, k, stride))


@pytest.mark.parametrize("h,w,k,stride", SHAPES)
def test_library_im2col_is_the_convolution(h, w, k, stride):
    import paper_2104_03152_amd as H
    rng = np.random.default_rng(h * 100 + w + 1)
    img = rng.uniform(0, 1, (h, w))
    kern = rng.normal(0, 1, (k, k))
    want = conv2d_direct(img, kern, stride)
    got = conv_via_im2col(H.he_im2col(img, k, stride), kern, h, w, k, stride)
    assert np.abs(got - want).max() < 1e-12


@pytest.mark.parametrize("h,w,k,stride", SHAPES)
@pytest.mark.parametrize("plant", ["offset", "window", "both"])
def test_planted_transposition_fails(h, w, k, stride, plant):
    rng = np.random.default_rng(7)
    img = rng.uniform(0, 1, (h, w))
    kern = rng.normal(0, 1, (k, k))
    bad = im2col_plain(img, k, stride, swap_offset=plant in ("offset", "both"),
                       swap_window=plant in ("window", "both"))
    got = conv_via_im2col(bad, kern, h, w, k, stride)
    assert np.abs(got - conv2d_direct(img, kern, stride)).max() > 1e-3


def test_direct_convolution_closed_forms():
    # a one-hot kernel picks one shifted, strided sub-image; a ones kernel
    # gives window sums (checked against cumulative sums)
    rng = np.random.default_rng(3)
    img = rng.uniform(0, 1, (11, 9))
    kern = np.zeros((4, 4))
    kern[1, 3] = 1.0
    assert np.array_equal(conv2d_direct(img, kern, 2), img[1:1 + 2 * 4:2, 3:3 + 2 * 3:2])
    c = np.pad(img.cumsum(0).cumsum(1), ((1, 0), (1, 0)))
    k = 3
    ws = c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]
    assert np.abs(conv2d_direct(img, np.ones((k, k)), 1) - ws).max() < 1e-12


def test_cnn_reference_uses_channel_major_packing():
    # FC1 input index c*64 + oy*8 + ox: with W1 selecting one input, the
    # network's hidden unit equals that channel's conv output at (oy, ox)
    rng = np.random.default_rng(4)
    d = {"img": rng.uniform(0, 1, (28, 28)), "conv_k": rng.normal(0, 0.1, (4, 49)),
         "conv_b": rng.normal(0, 0.1, 4), "w1": np.zeros((256, 64)), "b1": np.zeros(64),
         "w2": np.zeros((64, 10)), "b2": np.zeros(10)}
    c, oy, ox = 2, 5, 1
    d["w1"][c * 64 + oy * 8 + ox, 0] = 1.0
    d["w2"][0, 0] = 1.0
    conv = conv2d_direct(d["img"], d["conv_k"][c].reshape(7, 7), 3)[oy, ox] + d["conv_b"][c]
    assert abs(cnn_fp64(d)[0] - conv ** 4) < 1e-12
