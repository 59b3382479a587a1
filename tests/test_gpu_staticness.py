"""The static / dynamic split by staticness rho = beta / l (Sec. 3.2) on the
GPU against the oracle: bit-exact sizes, order and values, including the
empty input, all-static and all-dynamic thresholds, and a wrong output size
rejected before any write."""
import numpy as np
import pytest

import gen
from helpers import FIELDS, to_device

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,thr", [(1, 0.1), (257, 0.3), (50_000, 0.25), (3000, 1e9), (3000, 0.0)])
def test_split_bit_exact(orc, n, thr):
    import paper_2311_18561_amd as pvg
    sc = gen.make_scene(n, n % 97, sh_degree=3)
    st, dy = pvg.split_by_staticness(to_device(sc), thr)
    ref_s, ref_d = orc.adaptive.split_by_staticness(sc, thr)
    print(f"[split n={n} thr={thr}] static {ref_s['n']}, dynamic {ref_d['n']}")
    assert st[0].shape[-1] == ref_s["n"] and dy[0].shape[-1] == ref_d["n"]
    for f, a, b in zip(FIELDS, st, dy):
        assert np.array_equal(a.cpu().numpy(), ref_s[f]), f
        assert np.array_equal(b.cpu().numpy(), ref_d[f]), f


def test_split_empty_and_wrong_size():
    import ctypes as C

    import paper_2311_18561_amd as pvg
    from paper_2311_18561_amd import _lib as L
    from paper_2311_18561_amd.render import _p, gaussians_struct
    e = torch.empty
    empty = [e((3, 0)), e((3, 0)), e((4, 0)), e((16, 3, 0)), e((0,)), e((3, 0)), e((0,)), e((0,)), e((0,))]
    st, dy = pvg.split_by_staticness([t.cuda() for t in empty], 0.5)
    assert st[0].shape == (3, 0) and dy[0].shape == (3, 0)
    sc = gen.make_scene(1000, 3, sh_degree=3)
    params = to_device(sc)
    lib = L.load()
    size = C.c_size_t()
    L.check(lib.pvg_densify_tmp_bytes(1000, C.byref(size)))
    tmp = torch.empty(int(size.value), dtype=torch.uint8, device="cuda")
    g = gaussians_struct(params, 1000, 3)
    ns = C.c_int64()
    L.check(lib.pvg_staticness_split_plan(C.byref(g), 0.3, _p(tmp), int(tmp.numel()), C.byref(ns), None))
    m = int(ns.value)
    assert 0 < m < 1000
    a = [torch.empty((*p.shape[:-1], m + 1), device="cuda") for p in params]  # one too many
    b = [torch.empty((*p.shape[:-1], 1000 - m), device="cuda") for p in params]
    st = lib.pvg_staticness_split_apply(C.byref(g), 0.3, _p(tmp), int(tmp.numel()),
                                        C.byref(gaussians_struct(a, m + 1, 3)),
                                        C.byref(gaussians_struct(b, 1000 - m, 3)), None)
    assert st == -1
