"""Learned haptic-rate wrench surrogate around the SPH step (arXiv 2511.15908
Sec. 3.3): data collection through the SPH C ABI, feature rows, training and
haptic-tick inference through the MLP C ABI.  Argument marshalling and
bookkeeping only: the physics and the network run in libsph.so."""
from __future__ import annotations

import math

import numpy as np

from . import scenes

P_INIT = 40    # SplitMix64 purpose ids of the surrogate's random draws
P_BATCH = 41


def init_params(seed, hidden, layers, n_in, n_out):
    """LeCun-uniform initial weights (variance 1/fan_in over the real inputs),
    zero biases, padded rows and columns zero; flat parameter layout of
    include/sph_mlp.h."""
    rng = scenes.SplitMix64(seed, P_INIT)
    parts = []
    shapes = [(hidden, 128, n_in)] + [(hidden, hidden, hidden)] * (layers - 1) + [(16, hidden, hidden)]
    for li, (n, k, fan) in enumerate(shapes):
        a = math.sqrt(3.0 / fan)
        W = (2.0 * rng.uniform(n * k) - 1.0).reshape(n, k) * a
        W[:, fan:] = 0.0
        if li == len(shapes) - 1:
            W[n_out:] = 0.0
        parts += [W.ravel(), np.zeros(n)]
    return np.concatenate(parts).astype(np.float32)
