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
    # Transformer feed-forward block: N=2^16, 4 x 50-bit (FC, square, FC), dnum 2 (2 special), scale 2^40
    "ffn": (16, 4, 50, 2, 50, 2, 40, 3),
}

SEED_INPUT, SEED_WEIGHTS, SEED_ENC = 1, 2, 4

# hoisting mode of the benchmark configurations: 2, each layer's plan takes
# the schedule with the smaller modelled HBM traffic
BENCH_HOISTING = 2
# baby step of the convolutions' outer rotations: 0, chosen per layer by
# key-switch count (the plain form wherever C' <= 2, as in these networks)
BENCH_BABY_STEP = 0


def bench_config(fenc):
    """The benchmark configurations' per-layer schedule choices on a context."""
    fenc.set_hoisting(BENCH_HOISTING)
    fenc.set_baby_step(BENCH_BABY_STEP)
    return fenc


def images(shape, seed=SEED_INPUT):
    return np.random.default_rng(seed).uniform(0.0, 1.0, shape)


def weights(shapes, seed=SEED_WEIGHTS):
    r = np.random.default_rng(seed)
    return [r.normal(0.0, 0.1, s) for s in shapes]


LENET_SHAPES = [(6, 1, 5, 5), (16, 6, 5, 5), (120, 256), (84, 120), (10, 84)]
# the layer chain the block-size planner prices (the FC layers do not depend
# on the layout of their input and are left out)
LENET_LAYERS = [dict(kind="conv", cout=6, k=5), dict(kind="act"), dict(kind="pool"),
                dict(kind="conv", cout=16, k=5), dict(kind="act"), dict(kind="pool"), dict(kind="compress")]


def lenet_inputs(batch=64):
    """x[batch][1][28][28] and the five weight tensors of the LeNet-5-shaped network."""
    return images((batch, 1, 28, 28)), weights(LENET_SHAPES)


def planned_layout(fenc, batch, shape, layers):
    """Input layout at the block size the library's chain planner picks for
    `layers` (no repacks)."""
    S = fenc.plan_network(batch, shape, layers, 0)[0][0]
    c, h, w = shape
    return fenc.plan_layout(batch, c, h, w, layers[0]["k"], layers[0]["cout"], S)


def lenet_layout(fenc, batch=64):
    return planned_layout(fenc, batch, (1, 28, 28), LENET_LAYERS)


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


# CIFAR-shaped stack: 3 x (3x3 conv 16->16, same), 3x3 conv 16->32 stride 2,
# 3x3 conv 32->32 (same), a degree-3 polynomial activation after each conv
CIFAR_SHAPES = [(16, 16, 3, 3)] * 3 + [(32, 16, 3, 3), (32, 32, 3, 3)]
CIFAR_STRIDES = [1, 1, 1, 2, 1]
# a cubic of the ReLU-approximation kind (coefficients c0..c3)
CUBIC = (0.1, 0.5, 0.25, -0.02)


def cifar_inputs(batch=256, channels=16, side=32, shapes=None):
    """x[batch][channels][side][side] and the conv weights of the CIFAR-shaped stack."""
    return images((batch, channels, side, side)), weights(shapes or CIFAR_SHAPES)


def cifar_forward(fenc, ct, w, strides=None, coeffs=CUBIC):
    y = ct
    for wi, s in zip(w, strides or CIFAR_STRIDES):
        y = fenc.poly_act(fenc.conv2d(y, wi, stride=s, pad=wi.shape[2] // 2), coeffs, inplace=True)
    return y


# MobileNet-V1-shaped early blocks at ImageNet shape, each from a fresh encryption:
#   A: 3x3 conv 3->32 stride 2;  B: depthwise 3x3 (32) + pointwise 32->64;
#   C: depthwise 3x3 stride 2 (64) + pointwise 64->128;  a quadratic after each conv
MOBILENET_BLOCKS = [
    [dict(w=(32, 3, 3, 3), stride=2, pad=1, groups=1)],
    [dict(w=(32, 1, 3, 3), stride=1, pad=1, groups=32), dict(w=(64, 32, 1, 1), stride=1, pad=0, groups=1)],
    [dict(w=(64, 1, 3, 3), stride=2, pad=1, groups=64), dict(w=(128, 64, 1, 1), stride=1, pad=0, groups=1)],
]
# the input shape of each block's fresh encryption; its block size comes from
# the chain planner (mobilenet_layout)
MOBILENET_INPUTS = [(3, 224, 224), (32, 112, 112), (64, 112, 112)]
QUADRATIC = (0.1471, 0.5, 0.1196)   # a x^2 + b x + c of the ReLU-approximation kind


def mobilenet_weights(seed=SEED_WEIGHTS):
    return [weights([layer["w"] for layer in blk], seed=seed + i) for i, blk in enumerate(MOBILENET_BLOCKS)]


def mobilenet_layers(b):
    """Layer chain of block b for the planner."""
    out = []
    for ly in MOBILENET_BLOCKS[b]:
        out += [dict(kind="conv", cout=ly["w"][0], k=ly["w"][2], stride=ly["stride"], pad=ly["pad"],
                     groups=ly["groups"]), dict(kind="act")]
    return out


def mobilenet_layout(fenc, b, batch):
    return planned_layout(fenc, batch, MOBILENET_INPUTS[b], mobilenet_layers(b))


def mobilenet_encrypt(fenc, batch, seed_enc=SEED_ENC):
    """The three blocks' fresh encryptions of batch images each (the block
    inputs at 224x224x3, 112x112x32 and 112x112x64, uniform [0,1)), each at
    its planned block size."""
    cts = []
    for b, (c, h, w) in enumerate(MOBILENET_INPUTS):
        lay = mobilenet_layout(fenc, b, batch)
        cts.append(fenc.encrypt(fenc.encode_fragment(images((batch, c, h, w), seed=1 + b), lay), lay, seed_enc + b))
    return cts


def mobilenet_forward(fenc, cts, ws, coeffs=QUADRATIC):
    return [mobilenet_block(fenc, ct, blk, wb, coeffs) for ct, blk, wb in zip(cts, MOBILENET_BLOCKS, ws)]


# the single-layer configuration: one 28x28 image, conv 1->6 5x5 (valid)
CONV1_SHAPE = (6, 1, 5, 5)


def conv1_inputs(seed=SEED_INPUT):
    return images((1, 1, 28, 28), seed), weights([CONV1_SHAPE])[0]


def mobilenet_block(fenc, ct, blk, w, coeffs=QUADRATIC):
    """One block on an encrypted batch: each conv followed by the quadratic."""
    y = ct
    for layer, wi in zip(blk, w):
        # the activation overwrites the convolution's output buffer
        y = fenc.poly_act(fenc.conv2d(y, wi, stride=layer["stride"], pad=layer["pad"], groups=layer["groups"]),
                          coeffs, inplace=True)
    return y


# BERT-base-shaped feed-forward block on token fragments (the Transformer
# extension, Discussions): 128 tokens, E = 768 -> 3072 -> 768 with biases and
# a square activation between, embeddings split into S = 4 fragments
FFN_TOKENS, FFN_E, FFN_HIDDEN, FFN_S = 128, 768, 3072, 4


def ffn_inputs(n=FFN_TOKENS, E=FFN_E, H=FFN_HIDDEN, seed=SEED_INPUT):
    """x[n][E][1][1] uniform in [-1, 1) and (W1, b1, W2, b2) with N(0, 0.02)
    entries (BERT's initialisation scale)."""
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, (n, E, 1, 1))
    r = np.random.default_rng(seed + 1)
    return x, [r.normal(0.0, 0.02, s) for s in ((H, E), (H,), (E, H), (E,))]


def ffn_forward(fenc, ct, w):
    """FC E -> H (+ b1) -> x^2 -> FC H -> E (+ b2), on token fragments."""
    y = fenc.poly_act(fenc.fc(ct, w[0], bias=w[1]))
    return fenc.fc(y, w[2], bias=w[3])


def ffn_reference(x, w):
    n = x.shape[0]
    h = x.reshape(n, -1) @ w[0].T + w[1]
    return (h * h) @ w[2].T + w[3]
