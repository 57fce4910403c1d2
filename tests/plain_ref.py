"""Plaintext FP64 references for the convolution and the section 5 network,
written from their definitions and sharing nothing with either im2col
(oracle or library): the convolution slides the kernel over the image
window by window, so a transposed or mis-indexed im2col layout cannot agree
with it."""
import numpy as np


def conv2d_direct(img, kernel, stride):
    """Valid 2-D cross-correlation: out[oy, ox] = sum over (ky, kx) of
    img[oy*stride + ky, ox*stride + kx] * kernel[ky, kx] (section 3.2: the
    kernel applied to every window of the image)."""
    img = np.asarray(img, dtype=np.float64)
    kernel = np.asarray(kernel, dtype=np.float64)
    k = kernel.shape[0]
    assert kernel.shape == (k, k)
    h, w = img.shape
    oh, ow = (h - k) // stride + 1, (w - k) // stride + 1
    out = np.empty((oh, ow))
    for oy in range(oh):
        for ox in range(ow):
            win = img[oy * stride:oy * stride + k, ox * stride:ox * stride + k]
            out[oy, ox] = float((win * kernel).sum())
    return out


def cnn_fp64(d, img=None):
    """The section 5 network in plain FP64: 4 conv channels (7x7, stride 3)
    + bias, flattened channel-major (c*64 + oy*8 + ox, the packing order of
    the encrypted path), square, FC 256->64 + bias, square, FC 64->10 + bias."""
    img = d["img"] if img is None else img
    conv = np.stack([conv2d_direct(img, d["conv_k"][c].reshape(7, 7), 3) + d["conv_b"][c]
                     for c in range(d["conv_k"].shape[0])])
    x = conv.reshape(-1) ** 2
    h = (x @ d["w1"] + d["b1"]) ** 2
    return h @ d["w2"] + d["b2"]
