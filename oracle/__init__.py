"""Serial FP64 CPU oracle (ctypes wrapper around ``lsmg_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of ``bench.py`` may import this package; the GPU library and its Python
binding never do.  The oracle shares no code with the GPU path.

Vectors of a level are compact: ``[s-block | c-block]`` over the active nodes
ordered as inside nodes (lexicographic, x fastest) followed by ghost nodes
(lexicographic), the ordering map of section 3.3 (eq. maprij).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsmg_oracle.c")
_LIB = os.path.join(_HERE, "liblsmg_oracle.so")

OK, EINVAL, EGEOM, ENOCONV, ENONFINITE, EOOM = 0, -1, -2, -3, -4, -5


def build(force=True):
    """Compile the oracle with gcc (serial, -O2, no FMA contraction, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int), ("vcycles", ctypes.c_int),
                ("res_inf", ctypes.c_double), ("rho_last", ctypes.c_double),
                ("rho_geo", ctypes.c_double), ("dw_rel", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_L = ctypes.POINTER(ctypes.c_long)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    lib.or_build.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    lib.or_free.argtypes = [vp]
    lib.or_free.restype = None
    lib.or_set_params.argtypes = [vp] + [ctypes.c_double] * 7 + [ctypes.c_int] * 6 + [ctypes.c_double] + [ctypes.c_int] * 4
    lib.or_num_levels.argtypes = [vp]
    lib.or_level_info.argtypes = [vp, ctypes.c_int, _I, _D, _I, _I, _I]
    lib.or_compact_to_grid.argtypes = [vp, ctypes.c_int, _L]
    lib.or_ghost_table.argtypes = [vp, ctypes.c_int, _I, _D, _D, _D, _D, _I, _I]
    lib.or_set_linearization.argtypes = [vp, _D, ctypes.c_double]
    lib.or_apply_J.argtypes = [vp, ctypes.c_int, _D, _D]
    lib.or_smooth.argtypes = [vp, ctypes.c_int, _D, _D, ctypes.c_int]
    lib.or_defect.argtypes = [vp, ctypes.c_int, _D, _D, _D, _D]
    lib.or_restrict.argtypes = [vp, ctypes.c_int, _D, _D, _D]
    lib.or_band_nodes.argtypes = [vp, ctypes.c_int, _L]
    lib.or_prolong_add.argtypes = [vp, ctypes.c_int, _D, _D]
    lib.or_level_state.argtypes = [vp, ctypes.c_int, _D]
    lib.or_coarse_solve.argtypes = [vp, _D, _D]
    lib.or_vcycle.argtypes = [vp, ctypes.c_int, _D, _D, _D]
    lib.or_assemble_dense.argtypes = [vp, ctypes.c_int, _D]
    lib.or_assemble_coo.argtypes = [vp, ctypes.c_int, _I, _I, _D, _L]
    lib.or_residual.argtypes = [vp, _D, _D, ctypes.c_double, _D, _D, _D, _D, _D]
    lib.or_newton_cn_step.argtypes = [vp, _D, ctypes.c_double, _D, _D, _D, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(_Stats), _D, ctypes.c_int]
    lib.or_lu_solve_dense.argtypes = [_D, _D, ctypes.c_int]
    lib.or_krylov_solve.argtypes = [vp, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    lib.or_reinitialize.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _D]
    lib.or_levelset_from_mask.argtypes = [ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
    lib.or_extrapolate.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_double, _D, ctypes.c_int, _D]
    _lib = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def lu_solve_dense(A, b):
    """Dense LU with partial pivoting (the coarsest-grid solver), for its own pin."""
    lib = _load()
    A = _f64(A).copy()
    x = _f64(b).copy()
    _check(lib.or_lu_solve_dense(_dp(A), _dp(x), A.shape[0]), "lu")
    return x


def reinitialize(phi0, dim, n, h, iters):
    """Re-initialisation of a level set towards the signed distance (section 2)."""
    phi0 = _f64(phi0).reshape(-1)
    out = np.empty_like(phi0)
    _check(_load().or_reinitialize(_dp(phi0), dim, n, h, iters, _dp(out)), "reinitialize")
    return out


def levelset_from_mask(mask, dim, n, iters):
    """Level set -1 inside the mask, +1 outside, smoothed by iters heat steps (section 2)."""
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    out = np.empty(m.size)
    _check(_load().or_levelset_from_mask(m.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)), dim, n, iters, _dp(out)),
           "levelset_from_mask")
    return out


def extrapolate(phi, dim, n, h, q, iters):
    """Second-order extrapolation of q from phi < 0 to the rest of the grid (section 3.3)."""
    phi = _f64(phi).reshape(-1)
    q = _f64(q).reshape(-1)
    out = np.empty_like(q)
    _check(_load().or_extrapolate(_dp(phi), dim, n, h, _dp(q), iters, _dp(out)), "extrapolate")
    return out


class Hierarchy:
    """Level hierarchy of one domain: level 0 is the finest grid.  bc: boundary
    condition for s, 0 Dirichlet (eq. BCs) or 1 Neumann (section 3.6, eq. BCsN)."""

    def __init__(self, phi, dim, n, lo=-1.0, hi=1.0, coarsest_n=5, params=None, bc=0):
        lib = _load()
        phi = _f64(phi).reshape(-1)
        assert phi.size == n ** dim
        self._phi = phi
        h = ctypes.c_void_p()
        _check(lib.or_build(_dp(phi), dim, n, lo, hi, coarsest_n, int(bc), ctypes.byref(h)), "build")
        self._h = h
        self.dim, self.n, self.lo, self.hi, self.bc = dim, n, lo, hi, int(bc)
        self.nlev = lib.or_num_levels(h)
        self.params = dict(a=1e4, d=0.1, m_s=64.06, m_c=100.09, alpha=0.01, beta=0.1,
                           tau_s=0.9, nu1=2, nu2=2, ghost_c_new=1, band_steps=3,
                           ghost_sweeps=1, ghost_sweeps_coarse=None, sweeps_lambda=0.3, gamma=1, lex=0, fmg=0,
                           krylov_m=0)
        if params:
            self.set_params(**params)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_free(self._h)
            self._h = None

    def set_params(self, **kw):
        self.params.update(kw)
        p = self.params
        _check(_load().or_set_params(self._h, p["a"], p["d"], p["m_s"], p["m_c"], p["alpha"],
                                     p["beta"], p["tau_s"], int(p["nu1"]), int(p["nu2"]),
                                     int(p["ghost_c_new"]), int(p["band_steps"]),
                                     int(p["ghost_sweeps"]),
                                     int(p["ghost_sweeps"] if p["ghost_sweeps_coarse"] is None
                                         else p["ghost_sweeps_coarse"]),
                                     float(p["sweeps_lambda"]), int(p["gamma"]), int(p["lex"]),
                                     int(p["fmg"]), int(p["krylov_m"])), "set_params")

    # --- geometry ---------------------------------------------------------
    def level_info(self, l):
        n = ctypes.c_int(); h = ctypes.c_double(); ni = ctypes.c_int(); ng = ctypes.c_int()
        nb = ctypes.c_int()
        _check(_load().or_level_info(self._h, l, ctypes.byref(n), ctypes.byref(h), ctypes.byref(ni),
                                     ctypes.byref(ng), ctypes.byref(nb)), "level_info")
        return dict(n=n.value, h=h.value, ni=ni.value, ng=ng.value, na=ni.value + ng.value,
                    nb=nb.value)

    def compact_to_grid(self, l):
        info = self.level_info(l)
        out = np.zeros(info["na"], dtype=np.int64)
        _check(_load().or_compact_to_grid(self._h, l, out.ctypes.data_as(_L)), "c2g")
        return out

    def ghost_table(self, l):
        info = self.level_info(l)
        ng, nst, dim = info["ng"], 3 ** self.dim, self.dim
        st = np.zeros((ng, nst), dtype=np.int32)
        w = np.zeros((ng, nst)); B = np.zeros((ng, dim)); nrm = np.zeros((ng, dim))
        nrow = np.zeros((ng, dim))
        order = np.zeros(ng, dtype=np.int32); bfall = np.zeros(ng, dtype=np.int32)
        _check(_load().or_ghost_table(self._h, l, st.ctypes.data_as(_I), _dp(w), _dp(B), _dp(nrm),
                                      _dp(nrow), order.ctypes.data_as(_I), bfall.ctypes.data_as(_I)),
               "ghosts")
        return dict(st=st, w=w, B=B, normal=nrm, row_normal=nrow, order=order, bfallback=bfall)

    def band_nodes(self, l):
        info = self.level_info(l)
        out = np.zeros(info["nb"], dtype=np.int64)
        _check(_load().or_band_nodes(self._h, l, out.ctypes.data_as(_L)), "band")
        return out

    # --- grid <-> compact --------------------------------------------------
    def to_compact(self, l, s_grid, c_grid):
        idx = self.compact_to_grid(l)
        return np.concatenate([np.asarray(s_grid).reshape(-1)[idx], np.asarray(c_grid).reshape(-1)[idx]])

    def to_grid(self, l, v, fill=np.nan):
        info = self.level_info(l)
        idx = self.compact_to_grid(l)
        nn = info["n"] ** self.dim
        s = np.full(nn, fill); c = np.full(nn, fill)
        s[idx] = v[:info["na"]]; c[idx] = v[info["na"]:]
        return s, c

    # --- linear operators ---------------------------------------------------
    def set_linearization(self, W, dt):
        W = _f64(W)
        _check(_load().or_set_linearization(self._h, _dp(W), dt), "set_linearization")

    def level_state(self, l):
        out = np.zeros(2 * self.level_info(l)["na"])
        _check(_load().or_level_state(self._h, l, _dp(out)), "level_state")
        return out

    def apply_J(self, l, x):
        x = _f64(x); y = np.zeros_like(x)
        _check(_load().or_apply_J(self._h, l, _dp(x), _dp(y)), "apply_J")
        return y

    def smooth(self, l, rhs, x, nsweeps=1):
        rhs = _f64(rhs); x = _f64(x).copy()
        _check(_load().or_smooth(self._h, l, _dp(rhs), _dp(x), nsweeps), "smooth")
        return x

    def defect(self, l, rhs, x):
        rhs = _f64(rhs); x = _f64(x); r = np.zeros_like(x); nrm = ctypes.c_double()
        _check(_load().or_defect(self._h, l, _dp(rhs), _dp(x), _dp(r), ctypes.byref(nrm)), "defect")
        return r, nrm.value

    def restrict(self, l, r, return_band=False):
        r = _f64(r)
        rc = np.zeros(2 * self.level_info(l + 1)["na"])
        band = np.zeros(max(self.level_info(l)["nb"], 1))
        _check(_load().or_restrict(self._h, l, _dp(r), _dp(rc), _dp(band)), "restrict")
        if return_band:
            return rc, band[:self.level_info(l)["nb"]]
        return rc

    def prolong_add(self, l, ec, x):
        ec = _f64(ec); x = _f64(x).copy()
        _check(_load().or_prolong_add(self._h, l, _dp(ec), _dp(x)), "prolong")
        return x

    def coarse_solve(self, rhs):
        rhs = _f64(rhs); x = np.zeros_like(rhs)
        _check(_load().or_coarse_solve(self._h, _dp(rhs), _dp(x)), "coarse_solve")
        return x

    def vcycle(self, l, rhs, x):
        rhs = _f64(rhs); x = _f64(x).copy(); res = ctypes.c_double()
        _check(_load().or_vcycle(self._h, l, _dp(rhs), _dp(x), ctypes.byref(res)), "vcycle")
        return x, res.value

    def krylov_solve(self, F, m=30, rtol=1e-3, cycles_max=30):
        """Flexible GMRES(m) on level 0 at the current linearisation point, preconditioned
        by one V-cycle: returns (x, V-cycles taken)."""
        F = _f64(F); x = np.zeros_like(F)
        rc = _load().or_krylov_solve(self._h, _dp(F), _dp(x), int(m), float(rtol), int(cycles_max))
        if rc < 0:
            raise OracleError(rc, "krylov_solve")
        return x, rc

    def assemble_dense(self, l):
        N = 2 * self.level_info(l)["na"]
        A = np.zeros((N, N))
        _check(_load().or_assemble_dense(self._h, l, _dp(A)), "assemble_dense")
        return A

    def assemble_coo(self, l):
        info = self.level_info(l)
        cap = info["ni"] * (4 + 4 * self.dim) + info["ng"] * (3 ** self.dim + 2)
        rows = np.zeros(cap, dtype=np.int32); cols = np.zeros(cap, dtype=np.int32)
        vals = np.zeros(cap); nnz = ctypes.c_long(cap)
        _check(_load().or_assemble_coo(self._h, l, rows.ctypes.data_as(_I), cols.ctypes.data_as(_I),
                                       _dp(vals), ctypes.byref(nnz)), "assemble_coo")
        k = nnz.value
        return rows[:k], cols[:k], vals[:k]

    # --- Newton / Crank-Nicolson ---------------------------------------------
    def residual(self, W, Wn, dt, sb, fn=None, fnp1=None):
        W = _f64(W); Wn = _f64(Wn); sb = _f64(sb); fn = _f64(fn); fnp1 = _f64(fnp1)
        F = np.zeros_like(W); nrm = ctypes.c_double()
        _check(_load().or_residual(self._h, _dp(W), _dp(Wn), dt, _dp(sb), _dp(fn), _dp(fnp1),
                                   _dp(F), ctypes.byref(nrm)), "residual")
        return F, nrm.value

    def newton_cn_step(self, W, dt, sb, fn=None, fnp1=None, newton_tol=1e-10, newton_max=20,
                       lin_rtol=1e-3, cycles_max=30, rho_cap=0):
        """Returns (status, W_next, stats dict); W_next is W unchanged on failure."""
        W = _f64(W).copy(); sb = _f64(sb); fn = _f64(fn); fnp1 = _f64(fnp1)
        st = _Stats()
        rho = np.zeros(max(rho_cap, 1))
        rc = _load().or_newton_cn_step(self._h, _dp(W), dt, _dp(sb), _dp(fn), _dp(fnp1), newton_tol,
                                       newton_max, lin_rtol, cycles_max, ctypes.byref(st), _dp(rho),
                                       rho_cap)
        stats = dict(newton_iters=st.newton_iters, vcycles=st.vcycles, res_inf=st.res_inf,
                     rho_last=st.rho_last, rho_geo=st.rho_geo, dw_rel=st.dw_rel)
        if rho_cap:
            stats["rho"] = rho[:min(rho_cap, st.vcycles)].copy()
        return rc, W, stats
