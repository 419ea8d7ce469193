"""ctypes wrapper over the C oracle (test infrastructure only).

Each function mirrors one step of Zhang et al., "Binary Stereo Matching",
Section 3; the arithmetic lives in ``bsm_oracle.c``.  Arrays are numpy.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
INVALID_COST = 32767

_lib = None


def load():
    """Loads liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.path.join(HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    u8p = C.POINTER(C.c_uint8)
    i8p = C.POINTER(C.c_int8)
    u16p = C.POINTER(C.c_uint16)
    i16p = C.POINTER(C.c_int16)
    i32p = C.POINTER(C.c_int32)
    u64p = C.POINTER(C.c_uint64)
    ci = C.c_int
    lib.oracle_set_threads.argtypes = [ci]
    lib.oracle_get_threads.restype = ci
    lib.oracle_splitmix64_next.argtypes = [u64p]
    lib.oracle_splitmix64_next.restype = C.c_uint64
    lib.oracle_normal.argtypes = [u64p]
    lib.oracle_normal.restype = C.c_double
    lib.oracle_make_pattern.argtypes = [C.c_uint64, ci, ci, C.c_double, i8p]
    lib.oracle_make_pattern.restype = ci
    lib.oracle_luma.argtypes = [u8p, ci, ci, ci, u8p]
    lib.oracle_lab8_tables.argtypes = [u16p, i32p, u16p]
    lib.oracle_lab8.argtypes = [u8p, ci, ci, ci, u8p]
    lib.oracle_describe.argtypes = [u8p, ci, ci, ci, i8p, ci, u64p]
    lib.oracle_describe.restype = ci
    lib.oracle_weights.argtypes = [u8p, ci, ci, ci, i8p, ci, ci, ci, i32p]
    lib.oracle_weights.restype = ci
    lib.oracle_mask.argtypes = [u8p, ci, ci, ci, i8p, ci, ci, u64p, i32p]
    lib.oracle_mask.restype = ci
    lib.oracle_cost_volume.argtypes = [u64p, u64p, u64p, ci, ci, ci, ci, i16p]
    lib.oracle_cost_volume.restype = ci
    lib.oracle_wta.argtypes = [i16p, ci, ci, ci, i32p]
    lib.oracle_wta.restype = ci
    lib.oracle_match.argtypes = [u8p, u8p, ci, ci, ci, i8p, ci, ci, ci, ci,
                                 i32p, i16p]
    lib.oracle_match.restype = ci
    lib.oracle_match_right.argtypes = [u8p, u8p, ci, ci, ci, i8p, ci, ci, ci, ci, i32p, i16p]
    lib.oracle_match_right.restype = ci
    lib.oracle_lr_check.argtypes = [i32p, i32p, ci, ci, ci, i32p]
    lib.oracle_lr_check.restype = ci
    lib.oracle_vote_refine.argtypes = [u8p, ci, ci, ci, i32p, i32p, ci, ci, C.c_double, C.c_double,
                                       i32p, C.POINTER(C.c_double)]
    lib.oracle_vote_refine.restype = ci
    _lib = lib
    return lib


def _p(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def _img(img):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim != 3 or img.shape[2] != 3:
        raise ValueError("image must be HxWx3 uint8")
    H, W, _ = img.shape
    return img, W, H, 3 * W


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def set_threads(n):
    load().oracle_set_threads(int(n))


def get_threads():
    return load().oracle_get_threads()


def splitmix64(seed, count):
    """First ``count`` outputs of splitmix64 started at ``seed``."""
    st = C.c_uint64(seed)
    return [load().oracle_splitmix64_next(C.byref(st)) for _ in range(count)]


def normal_draws(seed, count):
    """``count`` Box-Muller standard normals from the splitmix64 stream."""
    lib = load()
    st = C.c_uint64(seed)
    return np.array([lib.oracle_normal(C.byref(st)) for _ in range(count)])


def make_pattern(seed, n, S, sigma):
    """int8 [n][4] = (px, py, qx, qy) offsets, Section 3 after Eq. 2."""
    out = np.zeros((n, 4), np.int8)
    _check(load().oracle_make_pattern(seed, n, S, float(sigma), _p(out, C.c_int8)),
           "make_pattern")
    return out


def luma(img):
    img, W, H, st = _img(img)
    out = np.zeros((H, W), np.uint8)
    load().oracle_luma(_p(img, C.c_uint8), W, H, st, _p(out, C.c_uint8))
    return out


def lab8_tables():
    lin = np.zeros(256, np.uint16)
    mq = np.zeros(9, np.int32)
    f = np.zeros(65536, np.uint16)
    load().oracle_lab8_tables(_p(lin, C.c_uint16), _p(mq, C.c_int32), _p(f, C.c_uint16))
    return lin, mq.reshape(3, 3), f


def lab8(img):
    img, W, H, st = _img(img)
    out = np.zeros((H, W, 3), np.uint8)
    load().oracle_lab8(_p(img, C.c_uint8), W, H, st, _p(out, C.c_uint8))
    return out


def _pat(pattern):
    pattern = np.ascontiguousarray(pattern, dtype=np.int8)
    if pattern.ndim != 2 or pattern.shape[1] != 4:
        raise ValueError("pattern must be [n][4] int8")
    return pattern, pattern.shape[0]


def describe(img, pattern):
    """uint64 [H][W][n/64] descriptors of Eq. 2-3."""
    img, W, H, st = _img(img)
    pattern, n = _pat(pattern)
    out = np.zeros((H, W, n // 64), np.uint64)
    _check(load().oracle_describe(_p(img, C.c_uint8), W, H, st, _p(pattern, C.c_int8),
                                  n, _p(out, C.c_uint64)), "describe")
    return out


def weights(img, pattern, u, v):
    """int32 [n] pair weights of Eq. 5 at pixel (u, v)."""
    img, W, H, st = _img(img)
    pattern, n = _pat(pattern)
    out = np.zeros(n, np.int32)
    _check(load().oracle_weights(_p(img, C.c_uint8), W, H, st, _p(pattern, C.c_int8),
                                 n, u, v, _p(out, C.c_int32)), "weights")
    return out


def mask(img, pattern, k=None):
    """(uint64 [H][W][n/64] mask of Eq. 6-7, int32 [H][W] threshold T)."""
    img, W, H, st = _img(img)
    pattern, n = _pat(pattern)
    k = n // 4 if k is None else int(k)
    out = np.zeros((H, W, n // 64), np.uint64)
    T = np.zeros((H, W), np.int32)
    _check(load().oracle_mask(_p(img, C.c_uint8), W, H, st, _p(pattern, C.c_int8), n,
                              k, _p(out, C.c_uint64), _p(T, C.c_int32)), "mask")
    return out, T


def cost_volume(descL, maskL, descR, dmax):
    """int16 [dmax][H][W] cost of Eq. 8 (Eq. 4 if maskL is None)."""
    descL = np.ascontiguousarray(descL, dtype=np.uint64)
    descR = np.ascontiguousarray(descR, dtype=np.uint64)
    if maskL is not None:
        maskL = np.ascontiguousarray(maskL, dtype=np.uint64)
    H, W, nw = descL.shape
    out = np.zeros((dmax, H, W), np.int16)
    _check(load().oracle_cost_volume(_p(descL, C.c_uint64), _p(maskL, C.c_uint64),
                                     _p(descR, C.c_uint64), W, H, nw * 64, dmax,
                                     _p(out, C.c_int16)), "cost_volume")
    return out


def wta(cost):
    """int32 [H][W] winner-take-all of Eq. 1, lowest d on ties."""
    cost = np.ascontiguousarray(cost, dtype=np.int16)
    dmax, H, W = cost.shape
    out = np.zeros((H, W), np.int32)
    _check(load().oracle_wta(_p(cost, C.c_int16), W, H, dmax, _p(out, C.c_int32)), "wta")
    return out


def match(left, right, pattern, dmax, k=None, use_mask=True, want_cost=False):
    """(disp int32 [H][W], cost int16 [dmax][H][W] or None) for one pair."""
    left, W, H, st = _img(left)
    right, W2, H2, _ = _img(right)
    if (W2, H2) != (W, H):
        raise ValueError("left and right must have the same shape")
    pattern, n = _pat(pattern)
    k = n // 4 if k is None else int(k)
    disp = np.zeros((H, W), np.int32)
    cost = np.zeros((dmax, H, W), np.int16) if want_cost else None
    _check(load().oracle_match(_p(left, C.c_uint8), _p(right, C.c_uint8), W, H, st,
                               _p(pattern, C.c_int8), n, k, 1 if use_mask else 0, dmax,
                               _p(disp, C.c_int32), _p(cost, C.c_int16)), "match")
    return disp, cost


def match_right(left, right, pattern, dmax, k=None, use_mask=True, want_cost=False):
    """Right-reference matching: (disp int32 [H][W] of the right view,
    cost int16 [dmax][H][W] or None), partner (u + d, v) in the left view."""
    left, W, H, st = _img(left)
    right, W2, H2, _ = _img(right)
    if (W2, H2) != (W, H):
        raise ValueError("left and right must have the same shape")
    pattern, n = _pat(pattern)
    k = n // 4 if k is None else int(k)
    disp = np.zeros((H, W), np.int32)
    cost = np.zeros((dmax, H, W), np.int16) if want_cost else None
    _check(load().oracle_match_right(_p(left, C.c_uint8), _p(right, C.c_uint8), W, H, st,
                                     _p(pattern, C.c_int8), n, k, 1 if use_mask else 0, dmax,
                                     _p(disp, C.c_int32), _p(cost, C.c_int16)), "match_right")
    return disp, cost


def lr_check(dL, dR, tol=1):
    """dL where |dL(u) - dR(u - dL(u))| <= tol, else -1."""
    dL = np.ascontiguousarray(dL, np.int32)
    dR = np.ascontiguousarray(dR, np.int32)
    if dL.shape != dR.shape or dL.ndim != 2:
        raise ValueError("dL and dR must be [H][W] of the same shape")
    H, W = dL.shape
    out = np.zeros((H, W), np.int32)
    _check(load().oracle_lr_check(_p(dL, C.c_int32), _p(dR, C.c_int32), W, H, int(tol),
                                  _p(out, C.c_int32)), "lr_check")
    return out


def vote_refine(rgb, checked, fallback, dmax, radius, lambda_c=9.0, lambda_e=16.0,
                want_votes=False):
    """Voting refinement of Eq. 9-10: (refined disparity int32 [H][W],
    W(x, d) float64 [H][W][dmax] of invalid pixels or None)."""
    rgb, W, H, st = _img(rgb)
    checked = np.ascontiguousarray(checked, np.int32)
    fallback = np.ascontiguousarray(fallback, np.int32)
    if checked.shape != (H, W) or fallback.shape != (H, W):
        raise ValueError("checked and fallback must be [H][W]")
    out = np.zeros((H, W), np.int32)
    votes = np.zeros((H, W, dmax), np.float64) if want_votes else None
    _check(load().oracle_vote_refine(_p(rgb, C.c_uint8), W, H, st, _p(checked, C.c_int32),
                                     _p(fallback, C.c_int32), int(radius), int(dmax),
                                     float(lambda_c), float(lambda_e), _p(out, C.c_int32),
                                     _p(votes, C.c_double)), "vote_refine")
    return out, votes
