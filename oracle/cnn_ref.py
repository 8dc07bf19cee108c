"""Float64 plaintext CNN used as the accuracy reference.  TEST INFRASTRUCTURE.

Evaluates eq. (multi-channel-conv) and the other layers of the encrypted
circuit directly on float64 tensors, so decrypted results can be compared
with the cleartext network (tolerance 1e-4 absolute at scale 2^40).
"""
import numpy as np


def conv2d(x, w, stride=1, pad=0, groups=1):
    """x[bs][cin][h][w], w[cout][cin/groups][k][k] -> [bs][cout][ho][wo] (cross-correlation)."""
    bs, cin, h, wd = x.shape
    cout, gin, k, _ = w.shape
    gout = cout // groups
    xp = np.zeros((bs, cin, h + 2 * pad, wd + 2 * pad))
    xp[:, :, pad:pad + h, pad:pad + wd] = x
    ho = (h + 2 * pad - k) // stride + 1
    wo = (wd + 2 * pad - k) // stride + 1
    y = np.zeros((bs, cout, ho, wo))
    for o in range(cout):
        g = o // gout
        for ci in range(gin):
            c = g * gin + ci
            for di in range(k):
                for dj in range(k):
                    y[:, o] += w[o, ci, di, dj] * xp[:, c, di:di + stride * ho:stride,
                                                     dj:dj + stride * wo:stride]
    return y


def avgpool2(x):
    bs, c, h, w = x.shape
    h2, w2 = h // 2, w // 2
    return x[:, :, :2 * h2, :2 * w2].reshape(bs, c, h2, 2, w2, 2).mean(axis=(3, 5))


def square(x):
    return x * x


def fc(x, w):
    """x[bs][...] flattened in C order, w[dout][din] -> [bs][dout][1][1]."""
    bs = x.shape[0]
    y = x.reshape(bs, -1) @ w.T
    return y.reshape(bs, -1, 1, 1)


def lenet(x, w1, w2, f1, f2, f3):
    """LeNet-5-shaped network of the benchmark: conv 5x5, x^2, avgpool, conv 5x5, x^2, avgpool, 3 FC."""
    y = avgpool2(square(conv2d(x, w1)))
    y = avgpool2(square(conv2d(y, w2)))
    return fc(fc(fc(y, f1), f2), f3)
