"""Python binding of the lsmg C ABI (``include/lsmg.h``): argument marshalling only.

Every computation runs in the HIP kernels of ``liblsmg.so``; PyTorch supplies
device memory (tensors' ``data_ptr()``) and the HIP stream.  The library must
have been built (``paper_1902_07029_amd.build.build()``); there is no fallback.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsmg.so")

OK, EINVAL, EGEOM, ENOCONV, ENONFINITE, EOOM, EHIP, ENOTIMPL = 0, -1, -2, -3, -4, -5, -6, -7
KERNEL_SMOOTH, KERNEL_DEFECT, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_GHOST = 0, 1, 2, 3, 4


class LsmgError(RuntimeError):
    def __init__(self, code, what, msg):
        super().__init__(f"{what} failed with status {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("d", ctypes.c_double), ("m_s", ctypes.c_double),
                ("m_c", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("tau_s", ctypes.c_double), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("ghost_sweeps", ctypes.c_int), ("ghost_sweeps_coarse", ctypes.c_int),
                ("band_steps", ctypes.c_int), ("ghost_c_new", ctypes.c_int),
                ("coarsest_n", ctypes.c_int), ("precision", ctypes.c_int), ("newton_tol", ctypes.c_double),
                ("newton_max", ctypes.c_int), ("lin_rtol", ctypes.c_double), ("cycles_max", ctypes.c_int),
                ("sweeps_lambda", ctypes.c_double), ("bc", ctypes.c_int), ("cycle_gamma", ctypes.c_int),
                ("fmg", ctypes.c_int), ("fused_sweep", ctypes.c_int),
                ("krylov_m", ctypes.c_int)]


class StepStats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("vcycles", ctypes.c_int), ("res_inf", ctypes.c_double),
                ("rho_last", ctypes.c_double), ("rho_geo", ctypes.c_double), ("dw_rel", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_vp = ctypes.c_void_p
_d = ctypes.c_double
_i = ctypes.c_int

_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp)
_FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp)


class Allocator(ctypes.Structure):
    """lsmg_allocator: device memory callbacks for the library's internal buffers."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", _vp)]


# one torch-backed allocator per stream; kept for the life of the process because
# hierarchies and batches hold its callbacks until they are destroyed
_TORCH_ALLOCATORS = {}


def torch_allocator(stream=None):
    """An lsmg_allocator backed by torch's caching allocator on `stream` (default:
    the current stream): the library's buffers then count in
    torch.cuda.memory_allocated() and share torch's pool."""
    stream = stream if stream is not None else torch.cuda.current_stream()
    key = (stream.device.index, stream.cuda_stream)
    if key in _TORCH_ALLOCATORS:
        return _TORCH_ALLOCATORS[key]
    dev = stream.device.index

    def _alloc(nbytes, _ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
        except Exception:      # out of memory: the library reports LSMG_EOOM
            return None

    def _free(ptr, _ctx):
        if ptr:
            torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)
    _TORCH_ALLOCATORS[key] = a
    return a


def load():
    """Load liblsmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_1902_07029_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    sigs = {
        "lsmg_default_params": (None, [ctypes.POINTER(Params)]),
        "lsmg_last_error": (ctypes.c_char_p, []),
        "lsmg_build_hierarchy": (_i, [_vp, ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.POINTER(Allocator),
                                      _vp, ctypes.POINTER(_vp)]),
        "lsmg_destroy_hierarchy": (None, [_vp]),
        "lsmg_set_params": (_i, [_vp, ctypes.POINTER(Params)]),
        "lsmg_set_dt": (_i, [_vp, _d]),
        "lsmg_get_params": (_i, [_vp, ctypes.POINTER(Params)]),
        "lsmg_num_levels": (_i, [_vp, ctypes.POINTER(_i)]),
        "lsmg_level_info": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_d), ctypes.POINTER(_i),
                                 ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "lsmg_compact_to_grid": (_i, [_vp, _i, _vp]),
        "lsmg_reinitialize": (_i, [_vp, _vp, _i, _vp]),
        "lsmg_reinitialize_noalloc": (_i, [_vp, _vp, _i, _vp]),
        "lsmg_levelset_from_mask": (_i, [_vp, _vp, _i, _vp, _vp]),
        "lsmg_extrapolate": (_i, [_vp, _vp, _vp, _i, _vp]),
        "lsmg_tail_in_lds": (_i, [_vp, _i, _vp]),
        "lsmg_sweep_fused": (_i, [_vp, _i, _i, _vp]),
        "lsmg_batch_sweep_fused": (_i, [_vp, _i, _i, _vp]),
        "lsmg_ghost_table": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "lsmg_state_create": (_i, [_vp, ctypes.POINTER(_vp)]),
        "lsmg_state_destroy": (None, [_vp]),
        "lsmg_state_set": (_i, [_vp, _vp]),
        "lsmg_state_get": (_i, [_vp, _vp]),
        "lsmg_state_set_grid": (_i, [_vp, _vp, _vp]),
        "lsmg_state_get_grid": (_i, [_vp, _vp, _vp]),
        "lsmg_newton_cn_step": (_i, [_vp, _vp, _d, _vp, _d, _vp, _vp, ctypes.POINTER(StepStats)]),
        "lsmg_residual": (_i, [_vp, _vp, _vp, _d, _vp, _d, _vp, _vp, _vp, ctypes.POINTER(_d)]),
        "lsmg_set_linearization": (_i, [_vp, _vp, _d]),
        "lsmg_level_state": (_i, [_vp, _i, _vp]),
        "lsmg_apply_J": (_i, [_vp, _i, _vp, _vp]),
        "lsmg_smooth": (_i, [_vp, _i, _vp, _vp, _i]),
        "lsmg_defect": (_i, [_vp, _i, _vp, _vp, _vp, ctypes.POINTER(_d)]),
        "lsmg_restrict": (_i, [_vp, _i, _vp, _vp]),
        "lsmg_prolong_add": (_i, [_vp, _i, _vp, _vp]),
        "lsmg_coarse_solve": (_i, [_vp, _vp, _vp]),
        "lsmg_vcycle": (_i, [_vp, _i, _vp, _vp, ctypes.POINTER(_d)]),
        "lsmg_profile_start": (_i, [_vp, _i, _i]),
        "lsmg_profile_stop": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
        "lsmg_memory_bytes": (_i, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "lsmg_estimate_bytes": (_i, [ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t)]),
        "lsmg_batch_create": (_i, [ctypes.POINTER(_vp), _i, ctypes.POINTER(Allocator), _vp, ctypes.POINTER(_vp)]),
        "lsmg_batch_destroy": (None, [_vp]),
        "lsmg_batch_step": (_i, [_vp, ctypes.POINTER(_vp), _d, ctypes.POINTER(_vp), ctypes.POINTER(_d),
                                 ctypes.POINTER(_i), ctypes.POINTER(StepStats)]),
        "lsmg_batch_set_autotune": (_i, [_vp, _i]),
        "lsmg_batch_advance": (_i, [_vp, ctypes.POINTER(_vp), _d, ctypes.POINTER(_d), ctypes.POINTER(_i), _i,
                                    ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(StepStats),
                                    ctypes.POINTER(_d), ctypes.POINTER(_i)]),
        "lsmg_batch_tuning": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "lsmg_batch_profile_start": (_i, [_vp, _i, _i]),
        "lsmg_batch_profile_stop": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return [n for n in dir(load()) if n.startswith("lsmg_")]


def _check(rc, what):
    if rc != OK:
        raise LsmgError(rc, what, load().lsmg_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


def _f64(t):
    assert t.dtype == torch.float64
    return _ptr(t)


def default_params(**overrides):
    p = Params()
    load().lsmg_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _stream(stream):
    return _vp(stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream)


def reinitialize(phi, dim, n, iterations, lo=-1.0, hi=1.0, stream=None):
    """Level set phi (CUDA float64, n^dim) re-initialised towards the signed distance, in place."""
    grid = Grid(dim, n, lo, hi)
    _check(load().lsmg_reinitialize(_ptr(phi), ctypes.byref(grid), iterations, _stream(stream)), "lsmg_reinitialize")
    return phi


def reinitialize_noalloc(phi, dim, n, iterations, lo=-1.0, hi=1.0, stream=None):
    """reinitialize() without any device allocation: the library's fixed scratch
    array (grids of up to 2^21 nodes; calls overlapping on one device race)."""
    grid = Grid(dim, n, lo, hi)
    _check(load().lsmg_reinitialize_noalloc(_ptr(phi), ctypes.byref(grid), iterations, _stream(stream)),
           "lsmg_reinitialize_noalloc")
    return phi


def levelset_from_mask(mask, dim, n, iterations, lo=-1.0, hi=1.0, stream=None):
    """Level set from a mask (CUDA uint8, n^dim; nonzero = inside): -1 / +1 smoothed by heat steps."""
    grid = Grid(dim, n, lo, hi)
    phi = torch.empty(mask.numel(), dtype=torch.float64, device=mask.device)
    _check(load().lsmg_levelset_from_mask(_ptr(mask), ctypes.byref(grid), iterations, _ptr(phi), _stream(stream)),
           "lsmg_levelset_from_mask")
    return phi


def extrapolate(phi, q, dim, n, iterations=40, lo=-1.0, hi=1.0, stream=None):
    """q (CUDA float64, n^dim) extrapolated from phi < 0 to every other node at second order, in place."""
    grid = Grid(dim, n, lo, hi)
    _check(load().lsmg_extrapolate(_ptr(phi), ctypes.byref(grid), _ptr(q), iterations, _stream(stream)),
           "lsmg_extrapolate")
    return q


def estimate_bytes(dim, n, params, lo=-1.0, hi=1.0):
    """(hierarchy bytes, state bytes) a hierarchy of this grid would hold (before building it)."""
    hb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    grid = Grid(dim, n, lo, hi)
    _check(load().lsmg_estimate_bytes(ctypes.byref(grid), ctypes.byref(params), ctypes.byref(hb), ctypes.byref(sb)),
           "lsmg_estimate_bytes")
    return hb.value, sb.value


class _Ordered:
    """Orders a library call that runs on `stream` with the caller's current stream:
    the library's stream first waits for the work queued on the current stream (the
    tensors passed in were written there), and the current stream then waits for the
    call's work (its outputs are read there).  Nothing to do when they are the same
    stream."""

    def __init__(self, stream):
        self.s = stream

    def __enter__(self):
        self.cur = torch.cuda.current_stream(self.s.device)
        if self.cur != self.s:
            self.s.wait_stream(self.cur)
        return self

    def __exit__(self, *exc):
        if self.cur != self.s:
            self.cur.wait_stream(self.s)
        return False


def _ordered(stream_of):
    def deco(fn):
        def wrapped(self, *a, **k):
            with _Ordered(stream_of(self)):
                return fn(self, *a, **k)
        wrapped.__name__, wrapped.__doc__ = fn.__name__, fn.__doc__
        return wrapped
    return deco


_own_stream = _ordered(lambda self: self.stream)
_hier_stream = _ordered(lambda self: self.hier.stream)


def _allocator_arg(allocator, stream):
    if allocator == "torch":
        return ctypes.byref(torch_allocator(stream))
    if allocator is None:
        return None
    return ctypes.byref(allocator)


class Hierarchy:
    """A domain's grid hierarchy on the current CUDA device and stream.  allocator:
    "torch" (default) takes the library's buffers from torch's caching allocator,
    None from hipMalloc, or an Allocator instance."""

    def __init__(self, phi, dim, n, lo=-1.0, hi=1.0, params=None, stream=None, allocator="torch"):
        lib = load()
        self.params = params if params is not None else default_params()
        self.dim, self.n, self.lo, self.hi = dim, n, lo, hi
        phi = phi.to(device="cuda", dtype=torch.float64).contiguous()
        assert phi.numel() == n ** dim
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        grid = Grid(dim, n, lo, hi)
        h = _vp()
        self._alloc = allocator
        _check(lib.lsmg_build_hierarchy(_f64(phi), ctypes.byref(grid), ctypes.byref(self.params),
                                        _allocator_arg(allocator, self.stream),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "lsmg_build_hierarchy")
        self._h = h
        nl = _i()
        _check(lib.lsmg_num_levels(h, ctypes.byref(nl)), "lsmg_num_levels")
        self.nlev = nl.value
        self.params = self.get_params()

    def get_params(self):
        p = Params()
        _check(load().lsmg_get_params(self._h, ctypes.byref(p)), "lsmg_get_params")
        return p

    def close(self):
        if getattr(self, "_h", None):
            load().lsmg_destroy_hierarchy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_dt(self, dt):
        """Prepare the hierarchy for time step dt (done by the first step otherwise)."""
        _check(load().lsmg_set_dt(self._h, dt), "lsmg_set_dt")

    def memory_bytes(self):
        """(hierarchy bytes, bytes of one state) on the device."""
        hb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().lsmg_memory_bytes(self._h, ctypes.byref(hb), ctypes.byref(sb)), "lsmg_memory_bytes")
        return hb.value, sb.value

    def set_params(self, params):
        _check(load().lsmg_set_params(self._h, ctypes.byref(params)), "lsmg_set_params")
        self.params = self.get_params()

    def level_info(self, l):
        n, h, ni, ng, nb = _i(), _d(), _i(), _i(), _i()
        _check(load().lsmg_level_info(self._h, l, ctypes.byref(n), ctypes.byref(h), ctypes.byref(ni),
                                      ctypes.byref(ng), ctypes.byref(nb)), "lsmg_level_info")
        return dict(n=n.value, h=h.value, ni=ni.value, ng=ng.value, na=ni.value + ng.value, nb=nb.value)

    def _vec(self, l):
        # an output the library writes in full (no fill kernel, which would race with a
        # library stream that has already been ordered after the current one)
        return torch.empty(2 * self.level_info(l)["na"], dtype=torch.float64, device="cuda")

    @_own_stream
    def compact_to_grid(self, l):
        out = torch.empty(self.level_info(l)["na"], dtype=torch.int64, device="cuda")
        _check(load().lsmg_compact_to_grid(self._h, l, _ptr(out)), "lsmg_compact_to_grid")
        return out

    def tail_in_lds(self, precision=0):
        v = _i()
        _check(load().lsmg_tail_in_lds(self._h, precision, ctypes.byref(v)), "lsmg_tail_in_lds")
        return bool(v.value)

    def sweep_fused(self, level, precision=0):
        v = _i()
        _check(load().lsmg_sweep_fused(self._h, level, precision, ctypes.byref(v)), "lsmg_sweep_fused")
        return bool(v.value)

    def tail_whole(self):
        """True when every level runs in the one-workgroup coarse tail (the finest level
        has at most 1024 active nodes)."""
        return self.level_info(0)["na"] <= 1024

    @_own_stream
    def ghost_table(self, l):
        info = self.level_info(l)
        ng, nst, dim = info["ng"], 3 ** self.dim, self.dim
        st = torch.empty((ng, nst), dtype=torch.int32, device="cuda")
        w = torch.empty((ng, nst), dtype=torch.float64, device="cuda")
        B = torch.empty((ng, dim), dtype=torch.float64, device="cuda")
        nrm = torch.empty((ng, dim), dtype=torch.float64, device="cuda")
        nrow = torch.empty((ng, dim), dtype=torch.float64, device="cuda")
        order = torch.empty(ng, dtype=torch.int32, device="cuda")
        bf = torch.empty(ng, dtype=torch.int32, device="cuda")
        _check(load().lsmg_ghost_table(self._h, l, _ptr(st), _ptr(w), _ptr(B), _ptr(nrm), _ptr(nrow), _ptr(order),
                                       _ptr(bf)), "lsmg_ghost_table")
        return dict(st=st, w=w, B=B, normal=nrm, row_normal=nrow, order=order, bfallback=bf)

    @_own_stream
    def residual(self, W, Wn, dt, sb=None, sb_const=1.0, fn=None, fnp1=None):
        F = torch.empty_like(W)
        nrm = _d()
        _check(load().lsmg_residual(self._h, _f64(W), _f64(Wn), dt, _ptr(sb), sb_const, _ptr(fn), _ptr(fnp1),
                                    _f64(F), ctypes.byref(nrm)), "lsmg_residual")
        return F, nrm.value

    @_own_stream
    def set_linearization(self, W, dt):
        _check(load().lsmg_set_linearization(self._h, _f64(W), dt), "lsmg_set_linearization")

    @_own_stream
    def level_state(self, l):
        out = self._vec(l)
        _check(load().lsmg_level_state(self._h, l, _f64(out)), "lsmg_level_state")
        return out

    @_own_stream
    def apply_J(self, l, x):
        y = torch.empty_like(x)
        _check(load().lsmg_apply_J(self._h, l, _f64(x), _f64(y)), "lsmg_apply_J")
        return y

    @_own_stream
    def smooth(self, l, rhs, x, nsweeps=1):
        x = x.clone()
        _check(load().lsmg_smooth(self._h, l, _f64(rhs), _f64(x), nsweeps), "lsmg_smooth")
        return x

    @_own_stream
    def defect(self, l, rhs, x):
        r = torch.empty_like(x)
        nrm = _d()
        _check(load().lsmg_defect(self._h, l, _f64(rhs), _f64(x), _f64(r), ctypes.byref(nrm)), "lsmg_defect")
        return r, nrm.value

    @_own_stream
    def restrict(self, l, r):
        rc = self._vec(l + 1)
        _check(load().lsmg_restrict(self._h, l, _f64(r), _f64(rc)), "lsmg_restrict")
        return rc

    @_own_stream
    def prolong_add(self, l, ec, x):
        x = x.clone()
        _check(load().lsmg_prolong_add(self._h, l, _f64(ec), _f64(x)), "lsmg_prolong_add")
        return x

    @_own_stream
    def coarse_solve(self, rhs):
        x = torch.empty_like(rhs)
        _check(load().lsmg_coarse_solve(self._h, _f64(rhs), _f64(x)), "lsmg_coarse_solve")
        return x

    def profile_start(self, kernel, level):
        _check(load().lsmg_profile_start(self._h, kernel, level), "lsmg_profile_start")

    def profile_stop(self):
        n, ms = _i(), _d()
        _check(load().lsmg_profile_stop(self._h, ctypes.byref(n), ctypes.byref(ms)), "lsmg_profile_stop")
        return n.value, ms.value

    @_own_stream
    def vcycle(self, l, rhs, x):
        x = x.clone()
        nrm = _d()
        _check(load().lsmg_vcycle(self._h, l, _f64(rhs), _f64(x), ctypes.byref(nrm)), "lsmg_vcycle")
        return x, nrm.value


class State:
    """W = (s, c) on the finest active nodes of a hierarchy."""

    def __init__(self, hier):
        self.hier = hier
        st = _vp()
        _check(load().lsmg_state_create(hier._h, ctypes.byref(st)), "lsmg_state_create")
        self._s = st

    def close(self):
        if getattr(self, "_s", None):
            load().lsmg_state_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @_hier_stream
    def set(self, W):
        _check(load().lsmg_state_set(self._s, _f64(W)), "lsmg_state_set")

    @_hier_stream
    def get(self):
        W = self.hier._vec(0)
        _check(load().lsmg_state_get(self._s, _f64(W)), "lsmg_state_get")
        return W

    @_hier_stream
    def set_grid(self, s, c):
        _check(load().lsmg_state_set_grid(self._s, _f64(s), _f64(c)), "lsmg_state_set_grid")

    @_hier_stream
    def get_grid(self):
        nn = self.hier.n ** self.hier.dim
        s = torch.empty(nn, dtype=torch.float64, device="cuda")
        c = torch.empty(nn, dtype=torch.float64, device="cuda")
        _check(load().lsmg_state_get_grid(self._s, _f64(s), _f64(c)), "lsmg_state_get_grid")
        return s, c

    @_hier_stream
    def step(self, dt, sb=None, sb_const=1.0, fn=None, fnp1=None, check=True):
        """One Crank-Nicolson step; returns (status, stats dict)."""
        st = StepStats()
        rc = load().lsmg_newton_cn_step(self.hier._h, self._s, dt, _ptr(sb), sb_const, _ptr(fn), _ptr(fnp1),
                                        ctypes.byref(st))
        if check:
            _check(rc, "lsmg_newton_cn_step")
        return rc, st.as_dict()


TUNE_CLASSES = ("smooth", "ghost", "defect", "restrict", "prolong", "band")


class Batch:
    """Hierarchies advanced together, one launch per kernel and grid size (lsmg_batch_*).

    The members (Hierarchy objects) must outlive the batch; they are kept
    referenced here."""

    def __init__(self, hierarchies, stream=None, autotune=True, allocator="torch"):
        lib = load()
        self.members = list(hierarchies)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (_vp * len(self.members))(*[h._h for h in self.members])
        b = _vp()
        self._alloc = allocator
        _check(lib.lsmg_batch_create(arr, len(self.members), _allocator_arg(allocator, self.stream),
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b)),
               "lsmg_batch_create")
        self._b = b
        if not autotune:
            _check(lib.lsmg_batch_set_autotune(b, 0), "lsmg_batch_set_autotune")

    def close(self):
        if getattr(self, "_b", None):
            load().lsmg_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @_own_stream
    def step(self, states, dt, sb=None, sb_const=None, check=True):
        """One Crank-Nicolson step of every member; returns (status list, stats list)."""
        n = len(self.members)
        assert len(states) == n
        st_arr = (_vp * n)(*[st._s for st in states])
        sb_arr = None
        if sb is not None:
            sb_arr = (_vp * n)(*[(t.data_ptr() if t is not None else None) for t in sb])
        sbc = None
        if sb_const is not None:
            sbc = (_d * n)(*sb_const)
        status = (_i * n)()
        stats = (StepStats * n)()
        rc = load().lsmg_batch_step(self._b, st_arr, dt, sb_arr, sbc, status, stats)
        if check:
            _check(rc, "lsmg_batch_step")
        return [status[k] for k in range(n)], [stats[k].as_dict() for k in range(n)]

    @_own_stream
    def advance(self, states, dt, remaining, sb_const=None, max_ticks=1 << 30):
        """Ticks at V-cycle granularity until some member ends a step; returns a list of
        (member, status, stats, step_ms) for the members whose step ended, and the ticks run."""
        n = len(self.members)
        st_arr = (_vp * n)(*[st._s for st in states])
        sbc = (_d * n)(*sb_const) if sb_const is not None else None
        rem = (_i * n)(*remaining)
        ended = (_i * n)()
        status = (_i * n)()
        stats = (StepStats * n)()
        ms = (_d * n)()
        ticks = _i()
        _check(load().lsmg_batch_advance(self._b, st_arr, dt, sbc, rem, max_ticks, ended, status, stats, ms,
                                         ctypes.byref(ticks)), "lsmg_batch_advance")
        out = [(k, status[k], stats[k].as_dict(), ms[k]) for k in range(n) if ended[k]]
        return out, ticks.value

    def tuning(self):
        """{grid size: {kernel class: wavefronts per workgroup}}."""
        cnt = _i()
        _check(load().lsmg_batch_tuning(self._b, 0, ctypes.byref(cnt), None, None), "lsmg_batch_tuning")
        m = cnt.value
        sizes = (_i * max(m, 1))()
        ipb = (_i * max(6 * m, 1))()
        _check(load().lsmg_batch_tuning(self._b, m, ctypes.byref(cnt), sizes, ipb), "lsmg_batch_tuning")
        return {sizes[z]: {c: ipb[6 * z + i] for i, c in enumerate(TUNE_CLASSES)} for z in range(m)}

    def sweep_fused(self, n, precision=0):
        v = _i()
        _check(load().lsmg_batch_sweep_fused(self._b, n, precision, ctypes.byref(v)), "lsmg_batch_sweep_fused")
        return bool(v.value)

    def profile_start(self, kernel, n):
        _check(load().lsmg_batch_profile_start(self._b, kernel, n), "lsmg_batch_profile_start")

    def profile_stop(self):
        n, ms = _i(), _d()
        _check(load().lsmg_batch_profile_stop(self._b, ctypes.byref(n), ctypes.byref(ms)), "lsmg_batch_profile_stop")
        return n.value, ms.value


class BatchGroup:
    """Members split into `groups` batches, each on its own stream and stepped from its
    own host thread, so that the batches' launch chains overlap on the device and one
    batch's host round trips hide behind the others' kernels.  Members are dealt
    largest first to the group with the fewest active nodes so far.  A member's results
    are those of its batch, which are bitwise those of the member alone."""

    def __init__(self, hierarchies, groups=4, autotune=True, allocator="torch"):
        import concurrent.futures
        self.members = list(hierarchies)
        groups = max(1, min(int(groups), len(self.members)))
        na = [h.level_info(0)["na"] for h in self.members]
        load_ = [0] * groups
        self.parts = [[] for _ in range(groups)]
        for k in sorted(range(len(self.members)), key=lambda k: -na[k]):
            g = min(range(groups), key=lambda g: load_[g])
            self.parts[g].append(k)
            load_[g] += na[k]
        self.parts = [sorted(p) for p in self.parts if p]
        self.streams = [torch.cuda.Stream() for _ in self.parts]
        self.batches = [Batch([self.members[k] for k in p], stream=s, autotune=autotune, allocator=allocator)
                        for p, s in zip(self.parts, self.streams)]
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=len(self.parts))
        self._first_done = False

    def close(self):
        for b in getattr(self, "batches", []):
            b.close()
        if getattr(self, "_pool", None):
            self._pool.shutdown(wait=True)
            self._pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, states, dt, check=True):
        """One Crank-Nicolson step of every member (states in member order); returns
        (status list, stats list) in member order."""
        n = len(self.members)
        assert len(states) == n

        def run(g):
            with torch.cuda.stream(self.streams[g]):
                return self.batches[g].step([states[k] for k in self.parts[g]], dt, check=check)

        status, stats = [None] * n, [None] * n
        if not self._first_done:
            # each batch times its launch shapes in its first step (the autotuner): the
            # batches take that step one after another, so no batch times its kernels
            # while another's run beside them
            results = [run(g) for g in range(len(self.parts))]
            self._first_done = True
        else:
            results = [f.result() for f in [self._pool.submit(run, g) for g in range(len(self.parts))]]
        for g, (sg, tg) in enumerate(results):
            for j, k in enumerate(self.parts[g]):
                status[k], stats[k] = sg[j], tg[j]
        return status, stats
