"""Thin ctypes binding of ``libhp.so`` (the C ABI declared in include/hp.h).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  The library must
have been built (``python -m paper_2311_02101_amd.build``); loading fails
loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhp.so")

HP_OK, HP_EINVAL, HP_ENOMEM, HP_EDEVICE, HP_EUNSUPPORTED = 0, -1, -2, -3, -4
HP_FP64, HP_FP32, HP_MIXED_BF16 = 0, 1, 2
PRECISION = {"f64": HP_FP64, "f32": HP_FP32, "mixed": HP_MIXED_BF16}
KERNEL = {"auto": 0, "pull": 1, "push": 2}

EXPORTS = ("hp_plan", "hp_run", "hp_run_noalloc", "hp_tune", "hp_check", "hp_plan_query", "hp_free",
           "hp_status_string", "hp_last_error", "hp_unit_propagate", "hp_merge_candidates", "hp_temper",
           "hp_get_temps", "hp_philox_xor")


class HpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class HpCnf(ct.Structure):
    _fields_ = [("n_formulas", ct.c_int32), ("var_offset", ct.POINTER(ct.c_int64)),
                ("clause_offset", ct.POINTER(ct.c_int64)), ("k", ct.c_int32),
                ("lits", ct.POINTER(ct.c_int32))]


class HpRbm(ct.Structure):
    _fields_ = [("k", ct.c_int32), ("l", ct.c_int32), ("n_temps", ct.c_int32),
                ("W", ct.POINTER(ct.c_double)), ("b", ct.POINTER(ct.c_double))]


class HpOpts(ct.Structure):
    _fields_ = [("chains", ct.c_int32), ("temp_of_chain", ct.POINTER(ct.c_int32)),
                ("precision", ct.c_int32), ("alpha", ct.c_double), ("seed", ct.c_uint64),
                ("threads", ct.c_int32), ("split", ct.c_int32), ("kernel", ct.c_int32),
                ("graph", ct.c_int32), ("size_rbms", ct.c_void_p), ("split_wait_limit", ct.c_int32)]


class HpPlanInfo(ct.Structure):
    _fields_ = [("threads", ct.c_int32), ("split", ct.c_int32), ("push_items", ct.c_int32),
                ("pull_items", ct.c_int32), ("fx_shift", ct.c_int32), ("n_buckets", ct.c_int32),
                ("lds_push", ct.c_int64), ("lds_pull", ct.c_int64),
                ("bucket_kind", ct.c_int32 * 16), ("bucket_items", ct.c_int32 * 16),
                ("bucket_threads", ct.c_int32 * 16), ("bucket_max_n", ct.c_int32 * 16),
                ("bucket_grid", ct.c_int32 * 16), ("bucket_dyn", ct.c_int32 * 16),
                ("forked", ct.c_int32)]


class HpState(ct.Structure):
    _fields_ = [("v", ct.c_void_p), ("nu", ct.c_void_p), ("s_max", ct.c_void_p),
                ("best", ct.c_void_p), ("t", ct.c_void_p), ("total_vars", ct.c_int64),
                ("n_formulas", ct.c_int32), ("chains", ct.c_int32), ("nu_bytes", ct.c_int32)]


_lib = None


def load():
    """Load libhp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2311_02101_amd.build` (no CPU fallback exists)")
    # Bind to the HIP runtime PyTorch already carries: torch loads its own
    # libamdhip64 (soname libamdhip64.so.7) by path, so importing it first
    # makes libhp.so's dependency resolve to that same copy.  Two runtimes in
    # one process would not share devices or streams.
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    lib.hp_plan.argtypes = [ct.POINTER(ct.c_void_p), ct.POINTER(HpCnf), ct.POINTER(HpRbm),
                            ct.POINTER(HpOpts), ct.c_void_p]
    lib.hp_plan.restype = ct.c_int
    lib.hp_run.argtypes = [ct.c_void_p, ct.POINTER(HpState), ct.c_int64, ct.c_void_p]
    lib.hp_run.restype = ct.c_int
    lib.hp_run_noalloc.argtypes = [ct.c_void_p, ct.POINTER(HpState), ct.c_int64, ct.c_void_p]
    lib.hp_run_noalloc.restype = ct.c_int
    lib.hp_tune.argtypes = [ct.c_void_p, ct.POINTER(HpState), ct.c_int64, ct.c_void_p]
    lib.hp_tune.restype = ct.c_int
    lib.hp_plan_query.argtypes = [ct.c_void_p, ct.POINTER(HpPlanInfo)]
    lib.hp_plan_query.restype = ct.c_int
    lib.hp_check.argtypes = [ct.c_void_p]
    lib.hp_check.restype = ct.c_int
    lib.hp_free.argtypes = [ct.c_void_p]
    lib.hp_free.restype = ct.c_int
    lib.hp_status_string.argtypes = [ct.c_int]
    lib.hp_status_string.restype = ct.c_char_p
    lib.hp_last_error.argtypes = []
    lib.hp_last_error.restype = ct.c_char_p
    lib.hp_unit_propagate.argtypes = [ct.POINTER(HpCnf), ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p, ct.c_int32]
    lib.hp_unit_propagate.restype = ct.c_int
    lib.hp_merge_candidates.argtypes = [ct.c_void_p, ct.POINTER(HpState), ct.c_void_p, ct.c_void_p]
    lib.hp_merge_candidates.restype = ct.c_int
    lib.hp_temper.argtypes = [ct.c_void_p, ct.POINTER(HpState), ct.c_int32, ct.c_void_p]
    lib.hp_temper.restype = ct.c_int
    lib.hp_get_temps.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
    lib.hp_get_temps.restype = ct.c_int
    lib.hp_philox_xor.argtypes = [ct.c_uint64, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32, ct.c_int64,
                                  ct.c_int64, ct.c_void_p, ct.c_void_p]
    lib.hp_philox_xor.restype = ct.c_int
    _lib = lib
    return lib


def unit_propagate(tables, n_vars, formula, v, nu, threads=0):
    """Prioritized unit propagation (host, ``hp_unit_propagate``) of the chains
    of one formula.  tables/n_vars: the formula batch; v: uint8 [B][N_f]; nu:
    float64 [B][N_f] (host arrays).  Returns the new uint8 [B][N_f]."""
    lib = load()
    tables = [np.asarray(t, dtype=np.int32) for t in tables]
    K = tables[0].shape[0]
    var_offset = np.concatenate([[0], np.cumsum([int(n) for n in n_vars])]).astype(np.int64)
    clause_offset = np.concatenate([[0], np.cumsum([t.shape[1] for t in tables])]).astype(np.int64)
    lits = np.ascontiguousarray(np.concatenate(tables, axis=1), dtype=np.int32)
    cnf = HpCnf(len(tables), _ptr(var_offset, ct.c_int64), _ptr(clause_offset, ct.c_int64), K,
                _ptr(lits, ct.c_int32))
    v = np.ascontiguousarray(v, dtype=np.uint8)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    if v.shape != nu.shape or v.ndim != 2 or v.shape[1] != int(n_vars[formula]):
        raise ValueError("v and nu must be [B][N_f] of the formula")
    out = np.empty_like(v)
    _check(lib.hp_unit_propagate(ct.byref(cnf), int(formula), v.shape[0], v.ctypes.data, nu.ctypes.data,
                                 out.ctypes.data, int(threads)))
    return out


def philox_xor(seed, formula, t, chain, phase, blocks, n_out, out, stream=None):
    """hp_philox_xor into the device uint32 tensor `out` ([n_out])."""
    _check(load().hp_philox_xor(int(seed) & (2 ** 64 - 1), int(formula), int(t), int(chain), int(phase),
                                int(blocks), int(n_out), ct.c_void_p(out.data_ptr()), _stream_handle(stream)))


def device_available() -> bool:
    import torch
    return torch.cuda.is_available()


def _check(status):
    if status != HP_OK:
        lib = load()
        raise HpError(status, f"{lib.hp_status_string(status).decode()}: "
                              f"{lib.hp_last_error().decode()}")


def _ptr(a, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class Plan:
    """A planned formula batch (``hp_plan``); call ``run`` with a ``State``.

    tables: list of per-formula signed 1-based [K][C_f] literal tables.
    n_vars: list of N_f.  W: [T][K][L], b: [T][L] canonical OR-gate RBMs.
    size_rbms: None, or the size-clustered model (Sec. 4): a dict K -> (W
    [T][K][L_K], b [T][L_K]) for K = 3 .. max(K, 3), L_K = 3 for K = 3 and
    K + 1 otherwise; each clause then uses the RBM of its own length.
    split_wait_limit: reloads of an exchanged word before a split workgroup
    gives up (0 = about a second); a tiny value forces the failure path."""

    def __init__(self, tables, n_vars, W, b, *, chains, temps=None, precision="f64",
                 alpha=1e-3, seed=0, threads=0, split=0, kernel="auto", graph=False,
                 stream=None, size_rbms=None, split_wait_limit=0):
        lib = load()
        tables = [np.asarray(t, dtype=np.int32) for t in tables]
        n_vars = [int(n) for n in n_vars]
        K = tables[0].shape[0]
        if any(t.shape[0] != K for t in tables):
            raise ValueError("all formulas must share the padded width K")
        W = np.ascontiguousarray(np.asarray(W, dtype=np.float64).reshape(-1, K, np.shape(W)[-1]))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(W.shape[0], W.shape[2]))
        self.K, self.L, self.T = K, W.shape[2], W.shape[0]
        self.F, self.B = len(tables), int(chains)
        self.n_vars = n_vars
        self.n_clauses = [t.shape[1] for t in tables]
        self.var_offset = np.concatenate([[0], np.cumsum(n_vars)]).astype(np.int64)
        self.clause_offset = np.concatenate([[0], np.cumsum(self.n_clauses)]).astype(np.int64)
        self.lits = np.ascontiguousarray(np.concatenate(tables, axis=1), dtype=np.int32)
        self.precision = precision
        cnf = HpCnf(self.F, _ptr(self.var_offset, ct.c_int64), _ptr(self.clause_offset, ct.c_int64),
                    K, _ptr(self.lits, ct.c_int32))
        rbm = HpRbm(K, self.L, self.T, _ptr(W, ct.c_double), _ptr(b, ct.c_double))
        tp = None
        if temps is not None:
            self.temps = np.ascontiguousarray(temps, dtype=np.int32)
            if self.temps.shape != (self.B,):
                raise ValueError("temps must have one entry per chain")
            tp = _ptr(self.temps, ct.c_int32)
        sr = None
        self.clustered = size_rbms is not None
        if size_rbms is not None:
            self._size_arrays = []
            sr = (HpRbm * 5)()
            for i, Kg in enumerate(range(3, max(K, 3) + 1)):
                Wg, bg = size_rbms[Kg]
                Lg = 3 if Kg == 3 else Kg + 1
                Wg = np.ascontiguousarray(np.asarray(Wg, dtype=np.float64).reshape(-1, Kg, Lg))
                bg = np.ascontiguousarray(np.asarray(bg, dtype=np.float64).reshape(Wg.shape[0], Lg))
                self._size_arrays += [Wg, bg]
                sr[i] = HpRbm(Kg, Lg, Wg.shape[0], _ptr(Wg, ct.c_double), _ptr(bg, ct.c_double))
            self._size_struct = sr
        opts = HpOpts(self.B, tp, PRECISION[precision], float(alpha), int(seed) & (2 ** 64 - 1),
                      int(threads), int(split), KERNEL[kernel], int(bool(graph)),
                      ct.cast(sr, ct.c_void_p) if sr is not None else None, int(split_wait_limit))
        h = ct.c_void_p()
        _check(lib.hp_plan(ct.byref(h), ct.byref(cnf), ct.byref(rbm), ct.byref(opts),
                           _stream_handle(stream)))
        self._h = h

    def info(self):
        """Launch configuration chosen by the library (dict)."""
        out = HpPlanInfo()
        _check(load().hp_plan_query(self._h, ct.byref(out)))
        d = {}
        nb = min(out.n_buckets, 16)
        for f, _ in HpPlanInfo._fields_:
            v = getattr(out, f)
            d[f] = list(v)[:nb] if f.startswith("bucket_") else v
        return d

    def tune(self, n_sweeps=5, stream=None):
        """Autotune the workgroup size of every launch on a scratch state."""
        scratch = self.new_state([np.zeros((self.B, n), np.uint8) for n in self.n_vars])
        _check(load().hp_tune(self._h, ct.byref(scratch.c_struct()), int(n_sweeps),
                              _stream_handle(stream)))
        return self.info()

    @property
    def split(self):
        """Workgroups per chain of the push launch."""
        return self.info()["split"]

    @property
    def total_vars(self):
        return int(self.var_offset[-1])

    def new_state(self, v0_list, device="cuda"):
        """Allocate a device state from per-formula [B][N_f] initial assignments
        (nu = 0.25, s_max = 0, best = v0, t = 0)."""
        return State.from_host(self, v0_list, device)

    def run(self, state, n_sweeps, stream=None):
        lib = load()
        _check(lib.hp_run(self._h, ct.byref(state.c_struct()), int(n_sweeps),
                          _stream_handle(stream)))

    def run_noalloc(self, state, n_sweeps, stream=None):
        """hp_run_noalloc: the same sweeps with the run's scratch in the
        library's static device array (allocates nothing)."""
        _check(load().hp_run_noalloc(self._h, ct.byref(state.c_struct()), int(n_sweeps),
                                     _stream_handle(stream)))

    def check(self):
        """Synchronise and raise if a split workgroup timed out waiting for the others."""
        _check(load().hp_check(self._h))

    def temper(self, state, parity, stream=None):
        """One replica-exchange round (``hp_temper``) on the pairs of one parity."""
        _check(load().hp_temper(self._h, ct.byref(state.c_struct()), int(parity), _stream_handle(stream)))

    def current_temps(self, stream=None):
        """Current temperature of every (formula, chain): int32 [F][B]."""
        out = np.empty((self.F, self.B), np.int32)
        _check(load().hp_get_temps(self._h, out.ctypes.data, _stream_handle(stream)))
        return out

    def merge_candidates(self, state, cand_v, stream=None):
        """Top-B merge (``hp_merge_candidates``) of candidate assignments
        (device uint8 tensor in the state's layout) into ``state``."""
        _check(load().hp_merge_candidates(self._h, ct.byref(state.c_struct()), ct.c_void_p(cand_v.data_ptr()),
                                          _stream_handle(stream)))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().hp_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class State:
    """Device chain state (torch tensors) in the layout of include/hp.h."""

    def __init__(self, plan, v, nu, s_max, best, t):
        self.plan, self.v, self.nu, self.s_max, self.best, self.t = plan, v, nu, s_max, best, t

    @classmethod
    def from_host(cls, plan, v0_list, device="cuda"):
        import torch
        flat = np.concatenate([np.asarray(v, dtype=np.uint8).reshape(-1) for v in v0_list])
        if flat.size != plan.total_vars * plan.B:
            raise ValueError("initial states do not match the plan's sizes")
        ndt = torch.float32 if plan.precision == "f32" else torch.float64
        v = torch.from_numpy(flat.copy()).to(device)
        nu = torch.full((flat.size,), 0.25, dtype=ndt, device=device)
        s_max = torch.zeros(plan.F * plan.B, dtype=torch.int32, device=device)
        best = v.clone()
        t = torch.zeros(1, dtype=torch.int64, device=device)
        return cls(plan, v, nu, s_max, best, t)

    def c_struct(self):
        p = self.plan
        return HpState(self.v.data_ptr(), self.nu.data_ptr(), self.s_max.data_ptr(),
                       self.best.data_ptr(), self.t.data_ptr(), p.total_vars, p.F, p.B,
                       self.nu.element_size())

    def formula(self, f, chains=None):
        """Host copies (v, nu, s_max, best) of formula f as [B][N_f] arrays
        (only the listed chains' rows if ``chains`` is given)."""
        p = self.plan
        a, n = int(p.var_offset[f]) * p.B, p.n_vars[f]
        sl = slice(a, a + n * p.B)
        out = (self.v[sl].cpu().numpy().reshape(p.B, n),
               self.nu[sl].cpu().numpy().reshape(p.B, n),
               self.s_max[f * p.B:(f + 1) * p.B].cpu().numpy().astype(np.int64),
               self.best[sl].cpu().numpy().reshape(p.B, n))
        if chains is not None:
            rows = np.asarray(chains, dtype=np.int64)
            out = tuple(x[rows] for x in out)
        return out

    def set_formula(self, f, v=None, nu=None, s_max=None, best=None, chains=None):
        """Overwrite the state of formula f ([B][N_f] arrays), or of the listed
        chains only ([len(chains)][N_f])."""
        import torch
        p = self.plan
        a, n = int(p.var_offset[f]) * p.B, p.n_vars[f]
        sl = slice(a, a + n * p.B)
        dev = self.v.device
        rows = slice(None) if chains is None else torch.as_tensor(np.asarray(chains, dtype=np.int64), device=dev)

        def put(dst, src, dtype):
            dst.view(p.B, -1)[rows] = torch.from_numpy(np.ascontiguousarray(src).reshape(-1, dst.numel() // p.B)).to(
                dev, dtype)
        if v is not None:
            put(self.v[sl], np.asarray(v, dtype=np.uint8), torch.uint8)
        if nu is not None:
            put(self.nu[sl], np.asarray(nu), self.nu.dtype)
        if s_max is not None:
            put(self.s_max[f * p.B:(f + 1) * p.B], np.asarray(s_max, dtype=np.int32), torch.int32)
        if best is not None:
            put(self.best[sl], np.asarray(best, dtype=np.uint8), torch.uint8)

    def set_t(self, t):
        self.t.fill_(int(t))

    def get_t(self):
        return int(self.t.item())
