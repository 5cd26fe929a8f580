"""Layer shapes and HE parameter sets of the five benchmark workloads.

Shapes follow the paper's evaluation networks (App. D: the MNIST MLP's first
layer 784->128, CIFAR-shaped 3x3 convolutions) and the batch sizes used for the
per-layer cost table (Table V, batch 64).  All convolutions are stride 1 with
"same" padding 1, which is the configuration the packed encodings of App. A
cover (a valid correlation over a zero-padded input).
"""
from dataclasses import dataclass, field
from typing import List, Tuple


@dataclass(frozen=True)
class LayerSpec:
    """One linear layer.  kind is "fc", "conv" (2-d) or "conv1d".

    FC layers are stored as conv layers with h = w = k = 1 and pad = 0: the
    matrix encoding of App. A is the 1x1 case of the convolution encoding.
    A Conv1d is the 2-d case with h = 1, a 1 x k kernel and padding along the
    length only (the paper evaluates Conv1d as such a specialisation).
    Weight layout is PyTorch's: fc (c_out, c_in), conv (c_out, c_in, k, k),
    conv1d (c_out, c_in, k).  Activations are (batch, c_in, h, w), fc
    (batch, c_in), conv1d (batch, c_in, w).  stride applies to both axes of a
    conv and to the length of a conv1d.
    """
    kind: str
    batch: int
    c_in: int
    c_out: int
    h: int = 1
    w: int = 1
    k: int = 1
    pad: int = 0
    stride: int = 1
    # value distributions, consumed by workloads.gen
    x_dist: Tuple = ("normal", 1.0)
    w_dist: Tuple = ("normal", 0.1)
    dy_dist: Tuple = ("normal", 1.0)
    # HE parameter set for this layer
    log2_n: int = 13
    num_limbs: int = 3
    prime_bits: int = 60

    @property
    def kh(self):
        return 1 if self.kind == "conv1d" else self.k

    @property
    def kw(self):
        return self.k

    @property
    def pad_h(self):
        return 0 if self.kind == "conv1d" else self.pad

    @property
    def pad_w(self):
        return self.pad

    @property
    def h_out(self):
        return (self.h + 2 * self.pad_h - self.kh) // self.stride + 1

    @property
    def w_out(self):
        return (self.w + 2 * self.pad_w - self.kw) // self.stride + 1

    def x_shape(self):
        if self.kind == "fc":
            return (self.batch, self.c_in)
        if self.kind == "conv1d":
            return (self.batch, self.c_in, self.w)
        return (self.batch, self.c_in, self.h, self.w)

    def w_shape(self):
        if self.kind == "fc":
            return (self.c_out, self.c_in)
        if self.kind == "conv1d":
            return (self.c_out, self.c_in, self.k)
        return (self.c_out, self.c_in, self.k, self.k)

    def y_shape(self):
        if self.kind == "fc":
            return (self.batch, self.c_out)
        if self.kind == "conv1d":
            return (self.batch, self.c_out, self.w_out)
        return (self.batch, self.c_out, self.h_out, self.w_out)


def fc(batch, c_in, c_out, **kw):
    return LayerSpec("fc", batch, c_in, c_out, **kw)


def conv(batch, c_in, c_out, hw, k=3, pad=1, **kw):
    return LayerSpec("conv", batch, c_in, c_out, hw, hw, k, pad, **kw)


def conv1d(batch, c_in, c_out, length, k=5, pad=0, **kw):
    return LayerSpec("conv1d", batch, c_in, c_out, 1, length, k, pad, **kw)


def he_std(fan_in):
    return (2.0 / fan_in) ** 0.5


@dataclass
class Config:
    index: int
    name: str
    layers: List[LayerSpec]
    ops: Tuple[str, ...]
    first_layer_shares: bool = False  # <X>_0 = 0 for the network's input layer
    seed: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


def _conv_he(batch, cin, cout, hw, log2_n, limbs):
    return conv(batch, cin, cout, hw, x_dist=("normal", 1.0), w_dist=("normal", he_std(cin * 9)),
                dy_dist=("normal", 1.0), log2_n=log2_n, num_limbs=limbs, prime_bits=60)


CONFIGS = {
    1: Config(1, "fc64x10_b8_fwd_n4096",
              [fc(8, 64, 10, x_dist=("normal", 1.0), w_dist=("normal", 0.1), log2_n=12, num_limbs=2,
                  prime_bits=50)],
              ops=("fwd",), first_layer_shares=True, seed=0),
    2: Config(2, "fc784x128_b64_fwdbwd_n8192",
              [fc(64, 784, 128, x_dist=("uniform", 0.0, 1.0), w_dist=("normal", 0.05),
                  dy_dist=("normal", 1.0), log2_n=13, num_limbs=3, prime_bits=60)],
              ops=("fwd", "dx", "dw"), seed=1),
    3: Config(3, "conv3x64_k3_32x32_b64_fwdbwd_n8192",
              [_conv_he(64, 3, 64, 32, 13, 3)],
              ops=("fwd", "dx", "dw"), seed=2),
    4: Config(4, "cnn4_b128_step_mixedN",
              [_conv_he(128, 3, 32, 32, 14, 4),
               _conv_he(128, 32, 64, 16, 13, 3),
               _conv_he(128, 64, 128, 8, 13, 3),
               fc(128, 2048, 10, x_dist=("normal", 1.0), w_dist=("normal", he_std(2048)),
                  dy_dist=("normal", 1.0), log2_n=14, num_limbs=4, prime_bits=60)],
              ops=("fwd", "dx", "dw"), seed=3),
    5: Config(5, "resnet8conv_b64_n16384",
              [_conv_he(64, 64, 64, 32, 14, 4)] * 3 + [_conv_he(64, 128, 128, 16, 14, 4)] * 3
              + [_conv_he(64, 256, 256, 8, 14, 4)] * 2,
              ops=("fwd", "dx", "dw"), seed=4),
}


# More layer shapes of the paper's evaluation networks (App. D, Table V), at
# batch 64: the MNIST CNN (its stride-2 5x5 convolution, then two FC layers),
# the AGNews TextCNN's two Conv1d layers (k = 5 over 256 x 64 and 128 x 30
# inputs), and Table V's largest FC layer 2048 -> 1001.
EXTRA_WORKLOADS = {
    "mnist_cnn_b64_n8192": Config(
        0, "mnist_cnn_b64_n8192",
        [conv(64, 1, 5, 28, k=5, pad=2, stride=2, x_dist=("uniform", 0.0, 1.0), w_dist=("normal", he_std(25)),
              log2_n=13, num_limbs=3, prime_bits=60),
         fc(64, 980, 100, x_dist=("normal", 1.0), w_dist=("normal", he_std(980)), log2_n=13, num_limbs=3,
            prime_bits=60),
         fc(64, 100, 10, x_dist=("normal", 1.0), w_dist=("normal", he_std(100)), log2_n=13, num_limbs=3,
            prime_bits=60)],
        ops=("fwd", "dx", "dw"), seed=6),
    "textcnn_b64_n8192": Config(
        0, "textcnn_b64_n8192",
        [conv1d(64, 256, 128, 64, k=5, x_dist=("normal", 1.0), w_dist=("normal", he_std(256 * 5)),
                log2_n=13, num_limbs=3, prime_bits=60),
         conv1d(64, 128, 128, 30, k=5, x_dist=("normal", 1.0), w_dist=("normal", he_std(128 * 5)),
                log2_n=13, num_limbs=3, prime_bits=60)],
        ops=("fwd", "dx", "dw"), seed=7),
    "fc2048x1001_b64_n8192": Config(
        0, "fc2048x1001_b64_n8192",
        [fc(64, 2048, 1001, x_dist=("normal", 1.0), w_dist=("normal", he_std(2048)), log2_n=13, num_limbs=3,
            prime_bits=60)],
        ops=("fwd", "dx", "dw"), seed=8),
}


def config_layers(index):
    return CONFIGS[index].layers


def small_cases():
    """Small layers spanning several tiles and ragged tails, for full
    ciphertext-level comparison (the oracle finishes them in seconds)."""
    return [
        fc(8, 64, 10, log2_n=12, num_limbs=2, prime_bits=50),
        fc(5, 37, 7, log2_n=11, num_limbs=2, prime_bits=50),
        conv(3, 2, 3, 5, k=3, pad=1, log2_n=11, num_limbs=2, prime_bits=50),
        conv(2, 3, 4, 7, k=3, pad=1, log2_n=11, num_limbs=3, prime_bits=60),
        conv(2, 2, 2, 6, k=2, pad=0, log2_n=10, num_limbs=2, prime_bits=60),
    ]
