"""Seeded synthetic workloads for the encrypted linear-layer product.

This package only draws numbers: layer shapes, HE parameter choices by name,
and seeded fixed-point tensors with the value distributions of the paper's
evaluation layers (MNIST/CIFAR-shaped FC and Conv2d layers, Sec. VI and
App. D).  It holds none of the method's arithmetic (no encodings, no HE), so
both the CPU oracle and the GPU path may import it.
"""
from .configs import LayerSpec, CONFIGS, EXTRA_WORKLOADS, config_layers, small_cases, fc, conv, conv1d  # noqa: F401
from .gen import (layer_tensors, config_tensors, uniform_residues, T_PLAIN, FRAC_BITS,  # noqa: F401
                  fixed_point, random_shares)
