"""Adam with bias correction (Kingma & Ba 2015), as used by the paper
(Sec. 3.6: beta1 = 0.9, beta2 = 0.999, eps = 1e-8; level-wise learning rate)
-- oracle.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading: the update is applied to the preconditioned gradient of Eq. 3, and
``step`` is the 1-based update count (epoch e -> step e + 1).
"""
from __future__ import annotations

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def update(theta, m, v, g, lr, step: int, beta1=BETA1, beta2=BETA2, eps=EPS):
    """One Adam update; returns (theta', m', v') in float64."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
