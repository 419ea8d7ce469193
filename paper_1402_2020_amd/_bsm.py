"""ctypes binding of libbsm.so (include/bsm.h).

The functions below carry the C names and only marshal arguments; every
step of the matching runs in the library's HIP kernels.  ``Context`` adds a
thin convenience layer that allocates outputs as torch CUDA tensors (torch is
used for device memory and streams only).
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsm.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ETOOBIG, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "BSM_OK", -1: "BSM_EINVAL", -2: "BSM_ENOMEM", -3: "BSM_EDEVICE",
                -4: "BSM_EAGAIN", -5: "BSM_ETOOBIG", -6: "BSM_ENOTFOUND"}
INVALID_COST = 32767

# Every symbol include/bsm.h declares.
EXPORTS = ("bsm_create", "bsm_destroy", "bsm_last_error", "bsm_make_pattern", "bsm_pattern",
           "bsm_footprint", "bsm_color", "bsm_describe", "bsm_describe_packed", "bsm_cost_wta", "bsm_match",
           "bsm_match_noalloc",
           "bsm_match_right", "bsm_lr_check", "bsm_vote_refine",
           "bsm_match_batch", "bsm_batch_stage_times", "bsm_get_tuning", "bsm_set_tuning",
           "bsm_autotune", "bsm_autotune_cached",
           "bsm_serve_config", "bsm_submit", "bsm_poll", "bsm_drain", "bsm_serve_stats")
# Every symbol include/bsm_peaks.h declares.
PEAK_EXPORTS = ("bsm_measure_peaks",)


class BsmError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {bsm_last_error()}")


class Params(C.Structure):
    _fields_ = [("n_bits", C.c_int32), ("window", C.c_int32), ("sigma", C.c_double),
                ("seed", C.c_uint64), ("pattern", C.POINTER(C.c_int8)),
                ("mask_rank", C.c_int32), ("use_mask", C.c_int32)]


class Pair(C.Structure):
    _fields_ = [("left", C.c_void_p), ("right", C.c_void_p), ("width", C.c_int32),
                ("height", C.c_int32), ("stride", C.c_int32), ("dmax", C.c_int32),
                ("disp", C.c_void_p), ("cost", C.c_void_p)]


class Times(C.Structure):
    _fields_ = [("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_start", C.c_double),
                ("t_end", C.c_double)]


class ServeCounters(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("groups", C.c_uint64), ("max_in_flight_bytes", C.c_uint64),
                ("max_group", C.c_int32), ("max_slots_busy", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Peaks(C.Structure):
    _fields_ = [("valu_int32_ops", C.c_double), ("valu_addxor_ops", C.c_double),
                ("mfma_i8_ops", C.c_double), ("mfma_fp4_ops", C.c_double),
                ("hbm_read_bps", C.c_double), ("hbm_copy_bps", C.c_double),
                ("compute_units", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Tuning(C.Structure):
    _fields_ = [("desc_tile_w", C.c_int32), ("cost_dchunk", C.c_int32),
                ("blocks_per_cu", C.c_int32 * 4), ("cost_mfma", C.c_int32),
                ("batch_tile_h", C.c_int32), ("pair_desc_th", C.c_int32),
                ("pair_right_px", C.c_int32), ("mfma_min_dmax", C.c_int32)]

    def as_dict(self):
        return {"desc_tile_w": self.desc_tile_w, "cost_dchunk": self.cost_dchunk,
                "blocks_per_cu": list(self.blocks_per_cu), "cost_mfma": self.cost_mfma,
                "batch_tile_h": self.batch_tile_h, "pair_desc_th": self.pair_desc_th,
                "pair_right_px": self.pair_right_px, "mfma_min_dmax": self.mfma_min_dmax}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.desc_tile_w = int(d["desc_tile_w"])
        t.cost_dchunk = int(d["cost_dchunk"])
        for i, v in enumerate(d.get("blocks_per_cu", [0, 0, 0, 0])):
            t.blocks_per_cu[i] = int(v)
        t.cost_mfma = int(d.get("cost_mfma", 1))
        t.batch_tile_h = int(d.get("batch_tile_h", 16))
        t.pair_desc_th = int(d.get("pair_desc_th", 0))
        t.pair_right_px = int(d.get("pair_right_px", 0))
        t.mfma_min_dmax = int(d.get("mfma_min_dmax", 17))
        return t


_lib = None


def load():
    """Loads libbsm.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, u64, sz = C.c_void_p, C.c_int32, C.c_uint64, C.c_size_t
    st = C.c_int
    sig = {
        "bsm_create": ([C.POINTER(Params), i32, C.POINTER(vp)], st),
        "bsm_destroy": ([vp], None),
        "bsm_last_error": ([], C.c_char_p),
        "bsm_make_pattern": ([u64, i32, i32, C.c_double, C.POINTER(C.c_int8)], st),
        "bsm_pattern": ([vp, C.POINTER(C.c_int8)], st),
        "bsm_footprint": ([vp, i32, i32, i32, i32], sz),
        "bsm_color": ([vp, vp, i32, i32, i32, vp, i32, vp], st),
        "bsm_describe": ([vp, vp, i32, i32, i32, vp, vp, vp], st),
        "bsm_describe_packed": ([vp, vp, i32, i32, vp, vp, vp], st),
        "bsm_cost_wta": ([vp, vp, vp, vp, i32, i32, i32, vp, vp, vp], st),
        "bsm_match": ([vp, vp, vp, i32, i32, i32, i32, vp, vp, vp], st),
        "bsm_match_noalloc": ([vp, vp, vp, i32, i32, i32, i32, vp, vp, vp], st),
        "bsm_match_right": ([vp, vp, vp, i32, i32, i32, i32, vp, vp, vp], st),
        "bsm_lr_check": ([vp, vp, vp, i32, i32, i32, vp, vp], st),
        "bsm_vote_refine": ([vp, vp, i32, i32, i32, vp, vp, i32, i32, C.c_float, C.c_float, vp, vp],
                            st),
        "bsm_match_batch": ([vp, C.POINTER(Pair), i32, vp], st),
        "bsm_batch_stage_times": ([vp, C.POINTER(Pair), i32, vp, C.POINTER(C.c_float)], st),
        "bsm_get_tuning": ([vp, C.POINTER(Tuning)], st),
        "bsm_set_tuning": ([vp, C.POINTER(Tuning)], st),
        "bsm_autotune": ([vp, C.POINTER(Pair), i32, i32, vp, C.POINTER(Tuning),
                          C.POINTER(C.c_double)], st),
        "bsm_autotune_cached": ([vp, C.POINTER(Pair), i32, i32, vp, C.c_char_p,
                                 C.POINTER(Tuning), C.POINTER(C.c_double), C.POINTER(i32)], st),
        "bsm_serve_config": ([vp, sz, i32, i32], st),
        "bsm_serve_stats": ([vp, C.POINTER(ServeCounters)], st),
        "bsm_submit": ([vp, C.POINTER(Pair), C.POINTER(u64)], st),
        "bsm_poll": ([vp, u64, C.POINTER(i32), C.POINTER(Times)], st),
        "bsm_drain": ([vp], st),
        "bsm_measure_peaks": ([i32, sz, i32, C.POINTER(Peaks)], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status, what):
    if status != OK:
        raise BsmError(status, what)


# ---- the C entry points, same names -------------------------------------

def bsm_last_error():
    return load().bsm_last_error().decode()


def bsm_make_pattern(seed, n, S, sigma):
    import numpy as np
    out = np.zeros((n, 4), np.int8)
    _check(load().bsm_make_pattern(seed, n, S, float(sigma),
                                   out.ctypes.data_as(C.POINTER(C.c_int8))), "bsm_make_pattern")
    return out


def bsm_create(n_bits, window, sigma=0.0, seed=0, pattern=None, mask_rank=0, use_mask=1,
               device=0):
    import numpy as np
    p = Params(n_bits, window, float(sigma), seed, None, mask_rank, int(use_mask))
    keep = None
    if pattern is not None:
        keep = np.ascontiguousarray(pattern, dtype=np.int8)
        p.pattern = keep.ctypes.data_as(C.POINTER(C.c_int8))
    h = C.c_void_p()
    _check(load().bsm_create(C.byref(p), device, C.byref(h)), "bsm_create")
    return h


def bsm_destroy(ctx):
    load().bsm_destroy(ctx)


def bsm_pattern(ctx, n):
    import numpy as np
    out = np.zeros((n, 4), np.int8)
    _check(load().bsm_pattern(ctx, out.ctypes.data_as(C.POINTER(C.c_int8))), "bsm_pattern")
    return out


def bsm_footprint(ctx, W, H, dmax, want_cost):
    return load().bsm_footprint(ctx, W, H, dmax, int(want_cost))


def bsm_color(ctx, img, W, H, stride, packed, want_lab, stream):
    return load().bsm_color(ctx, img, W, H, stride, packed, int(want_lab), stream)


def bsm_describe(ctx, img, W, H, stride, desc, mask, stream):
    return load().bsm_describe(ctx, img, W, H, stride, desc, mask, stream)


def bsm_describe_packed(ctx, packed, W, H, desc, mask, stream):
    return load().bsm_describe_packed(ctx, packed, W, H, desc, mask, stream)


def bsm_cost_wta(ctx, descL, maskL, descR, W, H, dmax, disp, cost, stream):
    return load().bsm_cost_wta(ctx, descL, maskL, descR, W, H, dmax, disp, cost, stream)


def bsm_match(ctx, left, right, W, H, stride, dmax, disp, cost, stream):
    return load().bsm_match(ctx, left, right, W, H, stride, dmax, disp, cost, stream)


def bsm_match_noalloc(ctx, left, right, W, H, stride, dmax, disp, cost, stream):
    return load().bsm_match_noalloc(ctx, left, right, W, H, stride, dmax, disp, cost, stream)


def bsm_match_right(ctx, left, right, W, H, stride, dmax, disp, cost, stream):
    return load().bsm_match_right(ctx, left, right, W, H, stride, dmax, disp, cost, stream)


def bsm_lr_check(ctx, disp_left, disp_right, W, H, tol, out, stream):
    return load().bsm_lr_check(ctx, disp_left, disp_right, W, H, tol, out, stream)


def bsm_vote_refine(ctx, left, W, H, stride, checked, fallback, dmax, radius, lambda_c, lambda_e,
                    out, stream):
    return load().bsm_vote_refine(ctx, left, W, H, stride, checked, fallback, dmax, radius,
                                  lambda_c, lambda_e, out, stream)


def bsm_match_batch(ctx, pairs, stream):
    arr = (Pair * len(pairs))(*pairs)
    return load().bsm_match_batch(ctx, arr, len(pairs), stream)


def bsm_get_tuning(ctx):
    t = Tuning()
    _check(load().bsm_get_tuning(ctx, C.byref(t)), "bsm_get_tuning")
    return t


def bsm_set_tuning(ctx, tuning):
    return load().bsm_set_tuning(ctx, C.byref(tuning))


def bsm_batch_stage_times(ctx, pairs, stream):
    """Returns (status, [colour, describe, cost, cost with volume] ms)."""
    arr = (Pair * len(pairs))(*pairs)
    ms = (C.c_float * 4)()
    st = load().bsm_batch_stage_times(ctx, arr, len(pairs), stream, ms)
    return st, list(ms)


def bsm_autotune(ctx, pairs, reps, stream):
    arr = (Pair * len(pairs))(*pairs)
    best = Tuning()
    ms = C.c_double()
    st = load().bsm_autotune(ctx, arr, len(pairs), reps, stream, C.byref(best), C.byref(ms))
    return st, best, ms.value


def bsm_autotune_cached(ctx, pairs, reps, stream, cache_path):
    arr = (Pair * len(pairs))(*pairs)
    best = Tuning()
    ms = C.c_double()
    hit = C.c_int32()
    path = None if cache_path is None else os.fsencode(cache_path)
    st = load().bsm_autotune_cached(ctx, arr, len(pairs), reps, stream, path, C.byref(best),
                                    C.byref(ms), C.byref(hit))
    return st, best, ms.value, bool(hit.value)


def bsm_serve_config(ctx, cap_bytes, max_queue, max_group=0):
    return load().bsm_serve_config(ctx, cap_bytes, max_queue, max_group)


def bsm_serve_stats(ctx):
    out = ServeCounters()
    st = load().bsm_serve_stats(ctx, C.byref(out))
    return st, out


def bsm_submit(ctx, pair):
    t = C.c_uint64()
    st = load().bsm_submit(ctx, C.byref(pair), C.byref(t))
    return st, t.value


def bsm_poll(ctx, ticket):
    state = C.c_int32()
    times = Times()
    st = load().bsm_poll(ctx, ticket, C.byref(state), C.byref(times))
    return st, state.value, times


def bsm_drain(ctx):
    return load().bsm_drain(ctx)


# ---- convenience layer over torch tensors --------------------------------

def bsm_measure_peaks(device=0, hbm_bytes=4 << 30, reps=3):
    """Measured vector-ALU, int8 and fp4 matrix and HBM rates of the device (dict)."""
    out = Peaks()
    _check(load().bsm_measure_peaks(device, hbm_bytes, reps, C.byref(out)), "bsm_measure_peaks")
    return out.as_dict()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """Owns a bsm_ctx.  Images are uint8 CUDA tensors [H][W][3]; descriptor
    and mask tensors are int64 [H][W][n/64] holding the uint64 words."""

    def __init__(self, n_bits, window, sigma=0.0, seed=0, pattern=None, mask_rank=0,
                 use_mask=True, device=0):
        self.n = n_bits
        self.nw = n_bits // 64
        self.window = window
        self._serving = {}  # ticket -> host arrays kept alive until reported
        self.device = device
        self.use_mask = bool(use_mask)
        self.h = bsm_create(n_bits, window, sigma, seed, pattern, mask_rank, use_mask, device)

    def close(self):
        if self.h is not None:
            bsm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pattern(self):
        return bsm_pattern(self.h, self.n)

    def footprint(self, W, H, dmax, want_cost=False):
        return bsm_footprint(self.h, W, H, dmax, want_cost)

    @staticmethod
    def _img(img):
        if img.dtype.itemsize != 1 or img.dim() != 3 or img.shape[2] != 3 or not img.is_cuda:
            raise ValueError("image must be a uint8 CUDA tensor [H][W][3]")
        img = img.contiguous()
        H, W, _ = img.shape
        return img, W, H, 3 * W

    def color(self, img, want_lab=True, stream=None):
        import torch
        img, W, H, st = self._img(img)
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
        _check(bsm_color(self.h, _ptr(img), W, H, st, _ptr(out), want_lab, _stream(stream)),
               "bsm_color")
        return out

    def describe(self, img, with_mask=False, stream=None):
        import torch
        img, W, H, st = self._img(img)
        desc = torch.empty((H, W, self.nw), dtype=torch.int64, device=img.device)
        mask = torch.empty_like(desc) if with_mask else None
        _check(bsm_describe(self.h, _ptr(img), W, H, st, _ptr(desc), _ptr(mask),
                            _stream(stream)), "bsm_describe")
        return desc, mask

    def describe_packed(self, packed, with_mask=False, stream=None):
        import torch
        H, W = packed.shape
        desc = torch.empty((H, W, self.nw), dtype=torch.int64, device=packed.device)
        mask = torch.empty_like(desc) if with_mask else None
        _check(bsm_describe_packed(self.h, _ptr(packed), W, H, _ptr(desc), _ptr(mask),
                                   _stream(stream)), "bsm_describe_packed")
        return desc, mask

    def cost_wta(self, descL, maskL, descR, dmax, want_cost=False, stream=None):
        import torch
        H, W, _ = descL.shape
        disp = torch.empty((H, W), dtype=torch.int32, device=descL.device)
        cost = torch.empty((dmax, H, W), dtype=torch.int16, device=descL.device) \
            if want_cost else None
        _check(bsm_cost_wta(self.h, _ptr(descL), _ptr(maskL), _ptr(descR), W, H, dmax,
                            _ptr(disp), _ptr(cost), _stream(stream)), "bsm_cost_wta")
        return disp, cost

    def match(self, left, right, dmax, want_cost=False, disp=None, cost=None, stream=None):
        import torch
        left, W, H, st = self._img(left)
        right, W2, H2, _ = self._img(right)
        if (W2, H2) != (W, H):
            raise ValueError("left and right must have the same shape")
        if disp is None:
            disp = torch.empty((H, W), dtype=torch.int32, device=left.device)
        if cost is None and want_cost:
            cost = torch.empty((dmax, H, W), dtype=torch.int16, device=left.device)
        _check(bsm_match(self.h, _ptr(left), _ptr(right), W, H, st, dmax, _ptr(disp),
                         _ptr(cost), _stream(stream)), "bsm_match")
        return disp, cost

    def match_noalloc(self, left, right, dmax, want_cost=False, disp=None, cost=None,
                      stream=None):
        """bsm_match with its scratch in the library's fixed device array
        (no allocation inside the call; outputs are allocated here unless
        given)."""
        import torch
        left, W, H, st = self._img(left)
        right, W2, H2, _ = self._img(right)
        if (W2, H2) != (W, H):
            raise ValueError("left and right must have the same shape")
        if disp is None:
            disp = torch.empty((H, W), dtype=torch.int32, device=left.device)
        if cost is None and want_cost:
            cost = torch.empty((dmax, H, W), dtype=torch.int16, device=left.device)
        _check(bsm_match_noalloc(self.h, _ptr(left), _ptr(right), W, H, st, dmax, _ptr(disp),
                                 _ptr(cost), _stream(stream)), "bsm_match_noalloc")
        return disp, cost

    def match_right(self, left, right, dmax, want_cost=False, disp=None, cost=None, stream=None):
        """Right-reference matching: disparities of the right view's pixels
        (partner (u + d, v) in the left view)."""
        import torch
        left, W, H, st = self._img(left)
        right, W2, H2, _ = self._img(right)
        if (W2, H2) != (W, H):
            raise ValueError("left and right must have the same shape")
        if disp is None:
            disp = torch.empty((H, W), dtype=torch.int32, device=left.device)
        if cost is None and want_cost:
            cost = torch.empty((dmax, H, W), dtype=torch.int16, device=left.device)
        _check(bsm_match_right(self.h, _ptr(left), _ptr(right), W, H, st, dmax, _ptr(disp),
                               _ptr(cost), _stream(stream)), "bsm_match_right")
        return disp, cost

    def lr_check(self, disp_left, disp_right, tol=1, out=None, stream=None):
        """disp_left where the two maps agree within tol, else -1."""
        import torch
        H, W = disp_left.shape
        if out is None:
            out = torch.empty_like(disp_left)
        _check(bsm_lr_check(self.h, _ptr(disp_left), _ptr(disp_right), W, H, tol, _ptr(out),
                            _stream(stream)), "bsm_lr_check")
        return out

    def vote_refine(self, left, checked, fallback, dmax, radius=None, lambda_c=9.0, lambda_e=16.0,
                    out=None, stream=None):
        """Voting refinement of the pixels `checked` marks invalid (< 0);
        radius defaults to half the matching window."""
        import torch
        left, W, H, st = self._img(left)
        if out is None:
            out = torch.empty((H, W), dtype=torch.int32, device=left.device)
        r = self.window // 2 if radius is None else radius
        _check(bsm_vote_refine(self.h, _ptr(left), W, H, st, _ptr(checked), _ptr(fallback), dmax,
                               r, lambda_c, lambda_e, _ptr(out), _stream(stream)),
               "bsm_vote_refine")
        return out

    def tuning(self):
        return bsm_get_tuning(self.h).as_dict()

    def set_tuning(self, d):
        _check(bsm_set_tuning(self.h, Tuning.from_dict(d)), "bsm_set_tuning")

    def autotune(self, items, reps=3, stream=None):
        """Times the batch path on items (list of (left, right, dmax)) for each
        candidate tuning and keeps the fastest; returns (tuning dict, ms)."""
        pairs, _, keep = self._pairs(items, False)
        st, best, ms = bsm_autotune(self.h, pairs, reps, _stream(stream))
        _check(st, "bsm_autotune")
        del keep
        return best.as_dict(), ms

    def autotune_cached(self, items, cache_path, reps=3, stream=None, want_cost=False):
        """As autotune, through the persistent cache at cache_path; returns
        (tuning dict, ms, hit)."""
        pairs, _, keep = self._pairs(items, want_cost)
        st, best, ms, hit = bsm_autotune_cached(self.h, pairs, reps, _stream(stream), cache_path)
        _check(st, "bsm_autotune_cached")
        del keep
        return best.as_dict(), ms, hit

    def _pairs(self, items, want_cost):
        import torch
        pairs, outs, keep = [], [], []
        for left, right, dmax in items:
            left, W, H, st = self._img(left)
            right, _, _, _ = self._img(right)
            disp = torch.empty((H, W), dtype=torch.int32, device=left.device)
            cost = torch.empty((dmax, H, W), dtype=torch.int16, device=left.device) \
                if want_cost else None
            keep += [left, right, disp, cost]
            outs.append((disp, cost))
            pairs.append(Pair(left.data_ptr(), right.data_ptr(), W, H, st, dmax,
                              disp.data_ptr(), None if cost is None else cost.data_ptr()))
        return pairs, outs, keep

    def match_batch(self, items, want_cost=False, stream=None):
        """items: list of (left, right, dmax) CUDA tensors; returns a list of
        (disp, cost)."""
        pairs, outs, keep = self._pairs(items, want_cost)
        _check(bsm_match_batch(self.h, pairs, _stream(stream)), "bsm_match_batch")
        return outs

    # ---- serving (host buffers) -------------------------------------------

    def serve_config(self, cap_bytes, max_queue, max_group=0):
        _check(bsm_serve_config(self.h, cap_bytes, max_queue, max_group), "bsm_serve_config")

    def serve_stats(self):
        st, out = bsm_serve_stats(self.h)
        _check(st, "bsm_serve_stats")
        return out.as_dict()

    def submit(self, left, right, dmax, want_cost=False):
        """Queues one pair of uint8 host arrays [H][W][3] (numpy); returns a
        ticket.  The arrays and the result buffers stay referenced here until
        the ticket is reported done or failed by poll()."""
        import numpy as np
        L = np.ascontiguousarray(left, dtype=np.uint8)
        R = np.ascontiguousarray(right, dtype=np.uint8)
        if L.ndim != 3 or L.shape[2] != 3 or R.shape != L.shape:
            raise ValueError("left and right must be uint8 arrays of the same shape [H][W][3]")
        H, W, _ = L.shape
        disp = np.empty((H, W), np.int32)
        cost = np.empty((dmax, H, W), np.int16) if want_cost else None
        pair = Pair(L.ctypes.data, R.ctypes.data, W, H, 3 * W, dmax, disp.ctypes.data,
                    None if cost is None else cost.ctypes.data)
        st, ticket = bsm_submit(self.h, pair)
        _check(st, "bsm_submit")
        self._serving[ticket] = (L, R, disp, cost)
        return ticket

    def poll(self, ticket):
        """Returns (state, times, (disp, cost) or None): state 0 pending,
        1 done, -1 failed; times = (arrive, admit, start, end) seconds."""
        st, state, t = bsm_poll(self.h, ticket)
        _check(st, "bsm_poll")
        times = (t.t_arrive, t.t_admit, t.t_start, t.t_end)
        if state == 0:
            return state, times, None
        _, _, disp, cost = self._serving.pop(ticket)
        return state, times, ((disp, cost) if state == 1 else None)

    def drain(self):
        _check(bsm_drain(self.h), "bsm_drain")
