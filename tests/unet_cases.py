"""Seeded network weights shared by the learned-preconditioner tests."""
import numpy as np

from oracle import unet


def random_weights(seed, head_scale=0.3, bias_scale=0.1):
    """He-scaled random weights, random biases, a scaled head; padding entries zero."""
    rng = np.random.default_rng(seed)
    offs, n = unet.layout()
    w = np.zeros(n)
    for (wo, bo), (cin, cout, taps) in zip(offs, unet.LAYERS):
        w[wo:bo] = rng.standard_normal(bo - wo) * np.sqrt(2.0 / (taps * cin))
        w[bo:bo + cout] = bias_scale * rng.standard_normal(cout)
    wo, bo = offs[8]
    w[wo:bo] *= head_scale
    return unet.mask_padding(w)
