"""Seeded synthetic workloads: parameter sets, input tensors and weights.

This module holds shapes and random inputs only (no homomorphic arithmetic);
the benchmark, the tests and the oracle-side checks draw their inputs from it.
Pixel values are uniform in [0, 1) and weights normal with standard deviation
0.1, standing in for MNIST / CIFAR-10 / ImageNet images and trained weights.
"""
import numpy as np

# (log_n, n_q, q_bits, n_p, p_bits, dnum, log2_scale, seed)
PARAMS = {
    # single conv layer, one 28x28 image: N=2^13, 4 x 40-bit + 1 special, scale 2^30
    "conv1_small": (13, 4, 40, 1, 40, 4, 30, 3),
    # LeNet-5-shaped network, 64 images: N=2^15, 20 x 50-bit, dnum 3 (7 special), scale 2^40
    "lenet": (15, 20, 50, 7, 50, 3, 40, 3),
    # CIFAR-shaped stack: N=2^16, 24 x 50-bit, dnum 4 (6 special), scale 2^40
    "cifar": (16, 24, 50, 6, 50, 4, 40, 3),
}

SEED_INPUT, SEED_WEIGHTS, SEED_ENC = 1, 2, 4


def images(shape, seed=SEED_INPUT):
    return np.random.default_rng(seed).uniform(0.0, 1.0, shape)


def weights(shapes, seed=SEED_WEIGHTS):
    r = np.random.default_rng(seed)
    return [r.normal(0.0, 0.1, s) for s in shapes]


LENET_SHAPES = [(6, 1, 5, 5), (16, 6, 5, 5), (120, 256), (84, 120), (10, 84)]


def lenet_inputs(batch=64):
    """x[batch][1][28][28] and the five weight tensors of the LeNet-5-shaped network."""
    return images((batch, 1, 28, 28)), weights(LENET_SHAPES)


def lenet_forward(fenc, ct, w):
    """conv 5x5 -> x^2 -> avgpool -> conv 5x5 -> x^2 -> avgpool -> compress -> 3 FC."""
    y = fenc.conv2d(ct, w[0])
    y = fenc.avgpool2(fenc.poly_act(y))
    y = fenc.conv2d(y, w[1])
    y = fenc.avgpool2(fenc.poly_act(y))
    y = fenc.compress(y)
    y = fenc.fc(y, w[2])
    y = fenc.fc(y, w[3])
    return fenc.fc(y, w[4])
