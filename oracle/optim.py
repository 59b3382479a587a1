"""Oracle of the optimizer step (Sec. 4: Adam with per-parameter learning
rates, and the opacity reset).

TEST INFRASTRUCTURE ONLY (see the package docstring).  FP64 numpy.  Adam as
Kingma and Ba define it (bias-corrected moments, eps added to the root of
the second), taken on each array in its unconstrained form: log of scale,
beta and l, logit of opacity, the values themselves for mean, quaternion,
SH, velocity and tau.  Pinned by ``tests/test_oracle_optim.py`` against
torch.optim.Adam on the CPU."""
from __future__ import annotations

import numpy as np

FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")
KIND = {"mu": "id", "scale": "log", "rot": "id", "sh": "id", "opacity": "logit", "vel": "id", "period": "log",
        "tau": "id", "beta": "log"}


def rows_of(sc):
    """(field, row index inside the field, flat row of the moments) in order."""
    out, r = [], 0
    for f in FIELDS:
        a = np.asarray(sc[f])
        k = a.size // int(sc["n"]) if sc["n"] else (1 if a.ndim == 1 else int(np.prod(a.shape[:-1])))
        for j in range(k):
            out.append((f, j, r))
            r += 1
    return out


def adam_step(sc, grads, m, v, lrs, t, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step; returns (new scene, m, v).  lrs: mu, scale, rot, sh0, shN,
    opacity, vel, period, tau, beta."""
    n = int(sc["n"])
    out = {k: (np.array(x, np.float64) if isinstance(x, np.ndarray) else x) for k, x in sc.items()}
    m, v = np.array(m, np.float64), np.array(v, np.float64)
    bc1, bc2 = 1.0 - beta1 ** t, 1.0 - beta2 ** t
    for f, j, r in rows_of(sc):
        p = out[f].reshape(-1, n)[j]
        g = np.asarray(grads[f], np.float64).reshape(-1, n)[j]
        kind = KIND[f]
        if kind == "log":
            raw, graw = np.log(p), g * p
        elif kind == "logit":
            raw, graw = np.log(p / (1.0 - p)), g * p * (1.0 - p)
        else:
            raw, graw = p.copy(), g
        m[r] = beta1 * m[r] + (1 - beta1) * graw
        v[r] = beta2 * v[r] + (1 - beta2) * graw * graw
        lr = lrs[f] if f != "sh" else (lrs["sh0"] if j < 3 else lrs["shN"])
        raw = raw - lr * (m[r] / bc1) / (np.sqrt(v[r] / bc2) + eps)
        new = np.exp(raw) if kind == "log" else (1.0 / (1.0 + np.exp(-raw)) if kind == "logit" else raw)
        out[f].reshape(-1, n)[j] = new if lr != 0 else p
    return out, m, v


def adam_dense(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step on a dense array taken as it is (the learnable sky cube
    map of Sec. 3.4); returns (new p, m, v), FP64."""
    p, g = np.asarray(p, np.float64), np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    bc1, bc2 = 1.0 - beta1 ** t, 1.0 - beta2 ** t
    new = p - lr * (m / bc1) / (np.sqrt(v / bc2) + eps) if lr != 0 else p.copy()
    return new, m, v
