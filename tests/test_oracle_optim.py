"""Pins of the Adam oracle: torch.optim.Adam (FP64, CPU) as the library
reference, on the values themselves and on the log / logit forms of the
constrained arrays (gradients chained by hand into that form, as the
step's definition says); the bias-corrected first step's closed form; a
zero rate leaves the value and still moves the moments."""
import numpy as np
import pytest

import gen
from oracle import optim as oo

torch = pytest.importorskip("torch")

LRS = {"mu": 4.8e-3, "scale": 5e-3, "rot": 1e-3, "sh0": 2.5e-3, "shN": 1.25e-4, "opacity": 0.005, "vel": 1e-3,
       "period": 0.0, "tau": 1e-3, "beta": 0.02}


def _scene(n=40, seed=0):
    sc = gen.make_scene(n, seed, sh_degree=1)
    return {k: (np.asarray(v, np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}


def _grads(sc, rng):
    return {f: rng.standard_normal(np.shape(sc[f])) * 1e-2 for f in oo.FIELDS}


def test_matches_torch_adam_in_each_form():
    sc = _scene()
    n = sc["n"]
    rng = np.random.default_rng(1)
    rows = oo.rows_of(sc)
    m = np.zeros((len(rows), n))
    v = np.zeros((len(rows), n))
    # torch side: one leaf per field in the optimizer's form
    form = {f: oo.KIND[f] for f in oo.FIELDS}
    to_raw = {"id": lambda p: p, "log": np.log, "logit": lambda p: np.log(p / (1 - p))}
    leaves = {f: torch.tensor(to_raw[form[f]](sc[f]), dtype=torch.float64, requires_grad=True) for f in oo.FIELDS}
    groups = []
    for f in oo.FIELDS:
        if f == "sh":
            continue
        groups.append({"params": [leaves[f]], "lr": LRS[f]})
    sh0 = torch.tensor(sc["sh"][:1], dtype=torch.float64, requires_grad=True)
    shN = torch.tensor(sc["sh"][1:], dtype=torch.float64, requires_grad=True)
    groups += [{"params": [sh0], "lr": LRS["sh0"]}, {"params": [shN], "lr": LRS["shN"]}]
    opt = torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-15)
    cur = sc
    for t in range(1, 4):
        g = _grads(sc, rng)
        cur, m, v = oo.adam_step(cur, g, m, v, LRS, t)
        for f in oo.FIELDS:
            if f == "sh":
                continue
            val = {"id": lambda x: x, "log": torch.exp, "logit": torch.sigmoid}[form[f]](leaves[f].detach())
            gt = torch.tensor(g[f])
            leaves[f].grad = gt * val if form[f] == "log" else (gt * val * (1 - val) if form[f] == "logit" else gt)
        sh0.grad, shN.grad = torch.tensor(g["sh"][:1]), torch.tensor(g["sh"][1:])
        opt.step()
        for f in oo.FIELDS:
            if f == "sh":
                ref = torch.cat([sh0.detach(), shN.detach()]).numpy()
            else:
                ref = {"id": lambda x: x, "log": torch.exp, "logit": torch.sigmoid}[form[f]](leaves[f].detach()).numpy()
            np.testing.assert_allclose(cur[f], ref, rtol=1e-12, atol=1e-14, err_msg=f"{f} step {t}")


def test_first_step_closed_form_and_zero_rate():
    """t = 1: m^ = g, v^ = g^2, so each value moves by lr sign(g) (eps
    aside); with a zero rate (the cycle length) the value stays and the
    moments still take (1 - beta) g and (1 - beta2) g^2."""
    sc = _scene(10, 2)
    n = sc["n"]
    rng = np.random.default_rng(2)
    g = _grads(sc, rng)
    rows = oo.rows_of(sc)
    out, m, v = oo.adam_step(sc, g, np.zeros((len(rows), n)), np.zeros((len(rows), n)), LRS, 1)
    np.testing.assert_allclose(out["mu"], sc["mu"] - LRS["mu"] * np.sign(g["mu"]), rtol=1e-12)
    np.testing.assert_allclose(out["tau"], sc["tau"] - LRS["tau"] * np.sign(g["tau"]), rtol=1e-12)
    np.testing.assert_allclose(np.log(out["scale"]), np.log(sc["scale"]) - LRS["scale"] * np.sign(g["scale"]),
                               rtol=1e-12)
    assert np.array_equal(out["period"], sc["period"])
    r_period = [r for f, j, r in rows if f == "period"][0]
    gl = g["period"] * sc["period"]
    np.testing.assert_allclose(m[r_period], 0.1 * gl, rtol=1e-12)
    np.testing.assert_allclose(v[r_period], 0.001 * gl * gl, rtol=1e-12)


def test_dense_adam_matches_torch_adam():
    """The cube-map step (a dense array as it is) against torch.optim.Adam
    over four steps, and its zero-rate case."""
    rng = np.random.default_rng(3)
    p0 = rng.uniform(0, 1, (6, 3, 5, 5))
    leaf = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([leaf], lr=2.5e-3, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0, np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 5):
        g = rng.standard_normal(p0.shape) * 1e-2
        g[0] = 0.0  # a face with no gradient keeps its texels
        p, m, v = oo.adam_dense(p, g, m, v, 2.5e-3, t)
        leaf.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(p, leaf.detach().numpy(), rtol=1e-12, atol=1e-15, err_msg=f"step {t}")
    assert np.array_equal(p[0], p0[0])
    q, m2, v2 = oo.adam_dense(p0, g, np.zeros_like(p0), np.zeros_like(p0), 0.0, 1)
    assert np.array_equal(q, p0)
    np.testing.assert_allclose(m2, 0.1 * g, rtol=1e-12)
    np.testing.assert_allclose(v2, 0.001 * g * g, rtol=1e-12)
