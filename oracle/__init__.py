"""CPU oracle of the PVG rasterizer (ctypes wrapper over ``pvg_oracle.cpp``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path never
does.  It shares no code with the GPU library.

Layouts follow the boundary's: parameters SoA ``[rows, N]``; images
``[3, H, W]``; per-Gaussian FP32 stage outputs ``xy [N,2]``, ``conic_op [N,4]``
(A, B, C, opacity at t), ``rgb [N,3]``, ``radius [N]``, ``rect [N,4]``,
``tiles [N]``, ``flags [N]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pvg_oracle.cpp")
# PVG_ORACLE_LIB: another build of pvg_oracle.cpp (an instrumented one, say)
_LIB = os.environ.get("PVG_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
FIELDS = ("mu", "scale", "rot", "sh", "opacity", "vel", "period", "tau", "beta")
from . import adaptive  # noqa: E402,F401  (adaptive control: numpy, no C)
from . import optim  # noqa: E402,F401  (Adam step: numpy, no C)
from . import ssim  # noqa: E402,F401  (SSIM loss term: numpy and scipy, no C)
TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (FP32 stays FP32: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _open(path):
    L = C.CDLL(path)
    vp = C.c_void_p
    i64, i32 = C.c_int64, C.c_int
    L.orc_preprocess_f32.argtypes = [i64, i32, vp, vp, i32, i32, vp] + [vp] * 9
    L.orc_preprocess_f32.restype = None
    L.orc_bin_sort.argtypes = [i64, vp, vp, vp, i32, i32, i64, vp, vp, vp]
    L.orc_bin_sort.restype = i64
    L.orc_render_f32.argtypes = [i64, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, i64, i64, vp, vp, vp, vp, vp,
                                 vp, vp]
    L.orc_render_f32.restype = None
    L.orc_render_margin_f32.argtypes = [i64, vp, vp, vp, vp, i32, i32, vp, vp, vp, i64, i64, vp, i32]
    L.orc_render_margin_f32.restype = None
    L.orc_render_bruteforce_f32.argtypes = [i64, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp]
    L.orc_render_bruteforce_f32.restype = None
    L.orc_render_f64.argtypes = [i64, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp, vp, vp, vp, vp]
    L.orc_render_f64.restype = C.c_double
    L.orc_backward_f64.argtypes = [i64, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                   vp, vp, vp, vp, vp, vp, vp]
    L.orc_backward_f64.restype = None
    L.orc_temporal_f64.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_double, i32, vp, vp]
    L.orc_temporal_f64.restype = None
    L.orc_sh_basis_f64.argtypes = [i32, vp, vp, vp]
    L.orc_sh_basis_f64.restype = None
    L.orc_project_f64.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp, vp]
    L.orc_project_f64.restype = C.c_int
    L.orc_sky_f64.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp, vp]
    L.orc_sky_f64.restype = None
    L.orc_sky_bwd_f64.argtypes = [vp, vp, vp, i32, vp, i32, i32, vp, vp, vp]
    L.orc_sky_bwd_f64.restype = None
    L.orc_sky_face_uv.argtypes = [vp, vp, vp]
    L.orc_sky_face_uv.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _open(_LIB)
    return _lib


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a variant of the oracle's source (the tests plant mistakes in
    it to show that a pin catches them) with the oracle's own flags."""
    src = out_path + ".cpp"
    with open(src, "w") as fh:
        fh.write(src_text)
    cmd = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-o",
           out_path, src]
    subprocess.run(cmd, check=True)
    return out_path


def source_text() -> str:
    with open(_SRC) as fh:
        return fh.read()


class use_library:
    """Context manager: every oracle call inside it goes to the library at
    `path` (a variant built by build_variant) instead of liboracle.so."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _open(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def cam_array(cam) -> np.ndarray:
    return np.concatenate([np.asarray(cam["R"], np.float32).reshape(9), np.asarray(cam["T"], np.float32),
                           np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["znear"]],
                                    np.float32)]).astype(np.float32)


def frame_array(t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    return np.array([t, dt, mode, bg[0], bg[1], bg[2]], np.float32)


def grid(cam):
    return (cam["width"] + TILE - 1) // TILE, (cam["height"] + TILE - 1) // TILE


def _param_ptrs(scene, dtype):
    arrs = [_c(scene[f], dtype) for f in FIELDS]
    ptrs = (C.c_void_p * 9)(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def preprocess_f32(scene, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0)) -> dict:
    n = int(scene["n"])
    arrs, ptrs = _param_ptrs(scene, np.float32)
    out = {
        "xy": np.zeros((n, 2), np.float32), "depth": np.zeros(n, np.float32),
        "conic_op": np.zeros((n, 4), np.float32), "rgb": np.zeros((n, 3), np.float32),
        "radius": np.zeros(n, np.int32), "rect": np.zeros((n, 4), np.int32),
        "tiles": np.zeros(n, np.uint32), "flags": np.zeros(n, np.uint32),
        "feat": np.zeros((n, 4), np.float32),  # mean velocity v~ (3) and staticness rho
    }
    cv, fv = cam_array(cam), frame_array(t, dt, mode, bg)
    lib().orc_preprocess_f32(n, int(scene["sh_degree"]), ptrs, _p(cv), cam["width"], cam["height"], _p(fv),
                             *[_p(out[k]) for k in ("xy", "depth", "conic_op", "rgb", "radius", "rect",
                                                    "tiles", "flags", "feat")])
    return out


def bin_sort(pre, cam) -> dict:
    n = pre["depth"].shape[0]
    GX, GY = grid(cam)
    M = int(pre["tiles"].astype(np.int64).sum())
    it = np.zeros(max(M, 1), np.uint32)
    ig = np.zeros(max(M, 1), np.uint32)
    ranges = np.zeros((GX * GY, 2), np.uint32)
    got = lib().orc_bin_sort(n, _p(pre["depth"]), _p(pre["rect"]), _p(pre["radius"]), GX, GY, M,
                             _p(it), _p(ig), _p(ranges))
    assert got == M, (got, M)
    return {"M": M, "inst_tile": it[:M], "inst_gauss": ig[:M], "ranges": ranges}


def render_f32(pre, bins, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0), tiles=None, want_depth=False,
               want_feat=False):
    """FP32 image, final_T and last contributor of the tiles [lo, hi); with
    want_depth also the blended depth channel sum T alpha z, and with
    want_feat the blended velocity and staticness maps [4,H,W] (appended)."""
    n = pre["depth"].shape[0]
    W, H = cam["width"], cam["height"]
    GX, GY = grid(cam)
    lo, hi = (0, GX * GY) if tiles is None else tiles
    img = np.zeros((3, H, W), np.float32)
    T = np.zeros((H, W), np.float32)
    nc = np.zeros((H, W), np.int32)
    cv, fv = cam_array(cam), frame_array(t, dt, mode, bg)
    ig = bins["inst_gauss"] if bins["M"] > 0 else np.zeros(1, np.uint32)
    D = np.zeros((H, W), np.float32) if want_depth else None
    F = np.zeros((4, H, W), np.float32) if want_feat else None
    lib().orc_render_f32(n, _p(pre["xy"]), _p(pre["conic_op"]), _p(pre["rgb"]), _p(pre["radius"]), _p(cv),
                         W, H, _p(fv), _p(bins["ranges"]), _p(ig), lo, hi, _p(img), _p(T), _p(nc),
                         _p(pre["depth"]), _p(D), _p(pre["feat"]), _p(F))
    out = (img, T, nc)
    if want_depth:
        out += (D,)
    if want_feat:
        out += (F,)
    return out


def render_margin_f32(pre, bins, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0), tiles=None, gradients=False):
    """Per-pixel decision margin of the FP32 walk over the tiles [lo, hi)
    (elsewhere +inf): below 1 some skip or stop decision of the pixel sits
    within the rounding a differently-rounded FP32 renderer may take the
    other way (see composite_pixel_f32 in the C source); with gradients also
    the adjoint's branch at the alpha clamp."""
    n = pre["depth"].shape[0]
    W, H = cam["width"], cam["height"]
    GX, GY = grid(cam)
    lo, hi = (0, GX * GY) if tiles is None else tiles
    m = np.full((H, W), np.inf, np.float32)
    fv = frame_array(t, dt, mode, bg)
    ig = bins["inst_gauss"] if bins["M"] > 0 else np.zeros(1, np.uint32)
    lib().orc_render_margin_f32(n, _p(pre["xy"]), _p(pre["conic_op"]), _p(pre["rgb"]), _p(pre["radius"]), W, H,
                                _p(fv), _p(bins["ranges"]), _p(ig), lo, hi, _p(m), 1 if gradients else 0)
    return m


def render_bruteforce_f32(pre, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0)):
    n = pre["depth"].shape[0]
    W, H = cam["width"], cam["height"]
    img = np.zeros((3, H, W), np.float32)
    T = np.zeros((H, W), np.float32)
    nc = np.zeros((H, W), np.int32)
    fv = frame_array(t, dt, mode, bg)
    lib().orc_render_bruteforce_f32(n, _p(pre["xy"]), _p(pre["depth"]), _p(pre["conic_op"]), _p(pre["rgb"]),
                                    _p(pre["radius"]), _p(pre["rect"]), W, H, _p(fv), _p(img), _p(T), _p(nc))
    return img, T, nc


def render(scene, cam, t, dt=0.0, mode=0, bg=(0.0, 0.0, 0.0)) -> dict:
    """The whole FP32 forward: preprocess, instances, per-pixel compositing."""
    pre = preprocess_f32(scene, cam, t, dt, mode, bg)
    bins = bin_sort(pre, cam)
    img, T, nc = render_f32(pre, bins, cam, t, dt, mode, bg)
    return {"pre": pre, "bins": bins, "img": img, "final_T": T, "n_contrib": nc}


def scene64(scene) -> dict:
    out = {"n": scene["n"], "sh_degree": scene["sh_degree"]}
    for f in FIELDS:
        out[f] = np.ascontiguousarray(scene[f], dtype=np.float64)
    return out


def render_f64(sc64, cam, t, dt, mode, bg, pre, bins, tile_mask=None, w=None, want_img=True, wD=None, wT=None,
               want_depth=False, wF=None, colour=None):
    """FP64 image on the FP32 stage's discrete structure; returns (sum(w*img)
    + sum(wD*depth) + sum(wT*final_T), img, final_T), and the depth channel
    as a fourth result with want_depth.  colour (optional, [N,3]): values
    composited in place of the SH colour (three channels of a per-Gaussian
    feature vector, Sec. 4.1)."""
    n = int(sc64["n"])
    W, H = cam["width"], cam["height"]
    arrs, ptrs = _param_ptrs(sc64, np.float64)
    img = np.zeros((3, H, W), np.float64) if want_img else None
    T = np.zeros((H, W), np.float64) if want_img else None
    cv, fv = cam_array(cam), frame_array(t, dt, mode, bg)
    ig = bins["inst_gauss"] if bins["M"] > 0 else np.zeros(1, np.uint32)
    wv = None if w is None else _c(w, np.float64)
    wDv = None if wD is None else _c(wD, np.float64)
    wTv = None if wT is None else _c(wT, np.float64)
    wFv = None if wF is None else _c(wF, np.float64)
    D = np.zeros((H, W), np.float64) if want_depth else None
    tm = None if tile_mask is None else _c(tile_mask, np.uint8)
    col = None if colour is None else _c(colour, np.float64)
    L = lib().orc_render_f64(n, int(sc64["sh_degree"]), ptrs, _p(cv), W, H, _p(fv), _p(pre["xy"]),
                             _p(pre["conic_op"]), _p(pre["radius"]), _p(pre["flags"]), _p(bins["ranges"]),
                             _p(ig), _p(tm), _p(wv), _p(img), _p(T), _p(wDv), _p(wTv), _p(D), _p(wFv), None,
                             _p(col))
    return (L, img, T, D) if want_depth else (L, img, T)


def normalized_depth_f64(depth, final_T):
    """Normalized depth of Sec. 3.1 per pixel: sum_i T_i alpha_i z_i / sum_i
    T_i alpha_i, from the blended depth (numerator) and final_T; the
    denominator is 1 - final_T, since the transmittances telescope (T_i alpha_i
    = T_i - T_(i+1)); 0 where no Gaussian contributes (the sum is then 0)."""
    A = 1.0 - np.asarray(final_T, np.float64)
    ok = A > 0.0
    return np.where(ok, np.asarray(depth, np.float64) / np.where(ok, A, 1.0), 0.0)


def normalized_depth_bwd_f64(g, depth, final_T):
    """Adjoint of normalized_depth_f64 for the upstream gradient g: returns
    (dD, dT), the gradients of the blended depth and of final_T.  Quotient
    rule on D / A with A = 1 - final_T: dD = g / A, dT = g (D / A) / A; both 0
    where A = 0."""
    A = 1.0 - np.asarray(final_T, np.float64)
    ok = A > 0.0
    ia = np.where(ok, 1.0 / np.where(ok, A, 1.0), 0.0)
    g = np.asarray(g, np.float64)
    return g * ia, g * (np.asarray(depth, np.float64) * ia) * ia


def backward_f64(sc64, cam, t, dt, mode, bg, pre, bins, dimg, tile_mask=None, dD=None, dT=None, dF=None,
                 colour=None, g2d_in=None, want_abs=False, want_terms=False):
    """FP64 gradients of sum(dimg * image) + sum(dD * depth) + sum(dT * final_T)
    + sum(dF * (velocity map, staticness map)) for every parameter array, and
    g2d [N,14] (entries 9..13: d depth, d v~, d rho).
    tile_mask (optional, one byte per tile): only these tiles are visited; dimg,
    dD and dT must be zero on every other tile.  g2d_in ([N,14]): skip the
    compositing adjoint and take these screen-space gradients through the
    chain rule.  want_abs: also return the per-Gaussian sums over the pixels of
    the absolute values of the screen-space terms ([N,14], third result).
    want_terms: instead return, third, per parameter entry the magnitude of
    its terms: those sums carried through the chain rule in absolute value
    (the scale an FP32 adjoint's rounding is relative to)."""
    n = int(sc64["n"])
    W, H = cam["width"], cam["height"]
    arrs, ptrs = _param_ptrs(sc64, np.float64)
    grads = {f: np.zeros_like(sc64[f], dtype=np.float64) for f in FIELDS}
    gptrs = (C.c_void_p * 9)(*[grads[f].ctypes.data for f in FIELDS])
    g2d = np.zeros((n, 14), np.float64)
    cv, fv = cam_array(cam), frame_array(t, dt, mode, bg)
    ig = bins["inst_gauss"] if bins["M"] > 0 else np.zeros(1, np.uint32)
    d = _c(dimg, np.float64)
    tm = None if tile_mask is None else _c(tile_mask, np.uint8)
    if tm is not None:
        GX, GY = grid(cam)
        assert tm.size == GX * GY
        keep = np.repeat(np.repeat(tm.reshape(GY, GX), 16, 0), 16, 1)[:H, :W].astype(bool)
        assert not np.any(d[:, ~keep]), "dimg must be zero outside the tile mask"
    dDv = None if dD is None else _c(dD, np.float64)
    dTv = None if dT is None else _c(dT, np.float64)
    dFv = None if dF is None else _c(dF, np.float64)
    col = None if colour is None else _c(colour, np.float64)  # feature values in place of the colour
    if tm is not None:
        if dFv is not None:
            assert not np.any(dFv[:, ~keep]), "dF must be zero outside the tile mask"
        for extra in (dDv, dTv):
            assert extra is None or not np.any(extra[~keep]), "dD and dT must be zero outside the tile mask"
    gin = None if g2d_in is None else _c(g2d_in, np.float64)
    g2a = np.zeros((n, 14), np.float64) if (want_abs or want_terms) else None
    terms = {f: np.zeros_like(sc64[f], dtype=np.float64) for f in FIELDS} if want_terms else None
    tptrs = (C.c_void_p * 9)(*[terms[f].ctypes.data for f in FIELDS]) if want_terms else None
    lib().orc_backward_f64(n, int(sc64["sh_degree"]), ptrs, _p(cv), W, H, _p(fv), _p(pre["xy"]),
                           _p(pre["conic_op"]), _p(pre["radius"]), _p(pre["flags"]), _p(bins["ranges"]),
                           _p(ig), _p(d), gptrs, _p(g2d), _p(tm), _p(dDv), _p(dTv), _p(dFv), _p(col), _p(gin),
                           _p(g2a), tptrs)
    if want_terms:
        return grads, g2d, terms
    return (grads, g2d, g2a) if want_abs else (grads, g2d)


def temporal_f64(mu, v, l, tau, beta, o, t, dt=0.0, mode=0):
    mu = _c(mu, np.float64)
    v = _c(v, np.float64)
    mu_r = np.zeros(3, np.float64)
    op = np.zeros(1, np.float64)
    lib().orc_temporal_f64(_p(mu), _p(v), l, tau, beta, o, t, dt, mode, _p(mu_r), _p(op))
    return mu_r, float(op[0])


def sh_basis_f64(direction, degree=3):
    d = _c(direction, np.float64)
    K = (degree + 1) ** 2
    Y = np.zeros(K, np.float64)
    dY = np.zeros((K, 3), np.float64)
    lib().orc_sh_basis_f64(degree, _p(d), _p(Y), _p(dY))
    return Y, dY


def project_f64(mu, s, q, cam):
    m = np.zeros(2, np.float64)
    J = np.zeros(4, np.float64)
    cov = np.zeros(3, np.float64)
    cv = cam_array(cam)
    mu, s, q = _c(mu, np.float64), _c(s, np.float64), _c(q, np.float64)  # held for the call
    lib().orc_project_f64(_p(mu), _p(s), _p(q), _p(cv), cam["width"], cam["height"], _p(m), _p(J), _p(cov))
    return m, J, cov


def sky_f64(img, opac, cube, cam, jitter=None):
    """Sky composite img + (1 - opac) f_sky(d) in FP64 (img [3,H,W], opac [H,W],
    cube [6,3,R,R], jitter optional [2,H,W] pixel offsets)."""
    W, H = cam["width"], cam["height"]
    R = int(cube.shape[-1])
    out = np.zeros((3, H, W), np.float64)
    cv = cam_array(cam)
    jv = None if jitter is None else _c(jitter, np.float32)
    img, opac, cube = _c(img, np.float64), _c(opac, np.float64), _c(cube, np.float64)  # held for the call
    lib().orc_sky_f64(_p(img), _p(opac), _p(cube), R, _p(cv), W, H, _p(jv), _p(out))
    return out


def sky_bwd_f64(g, opac, cube, cam, jitter=None):
    """Adjoint of sky_f64 for dL/dout = g: (dL/dopac [H,W], dL/dcube [6,3,R,R])."""
    W, H = cam["width"], cam["height"]
    R = int(cube.shape[-1])
    dO = np.zeros((H, W), np.float64)
    dC = np.zeros((6, 3, R, R), np.float64)
    cv = cam_array(cam)
    jv = None if jitter is None else _c(jitter, np.float32)
    g, opac, cube = _c(g, np.float64), _c(opac, np.float64), _c(cube, np.float64)  # held for the call
    lib().orc_sky_bwd_f64(_p(g), _p(opac), _p(cube), R, _p(cv), W, H, _p(jv), _p(dO), _p(dC))
    return dO, dC


def sky_face_uv(d):
    face = np.zeros(1, np.int32)
    uv = np.zeros(2, np.float64)
    d = _c(d, np.float64)
    lib().orc_sky_face_uv(_p(d), _p(face), _p(uv))
    return int(face[0]), uv
