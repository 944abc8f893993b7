"""Python binding of libhsim.so: argument marshalling only.

Every ``hsim_*`` function here calls the C entry point of the same name
(include/hsim.h); the classes below only allocate torch device memory for the
buffers the library asks for and pass pointers and the current HIP stream.
All computation runs in the library's HIP kernels.  If the library or a GPU is
missing, the calls raise; there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HSIM_LIBRARY", os.path.join(_HERE, "libhsim.so"))

FP32, FP64_EXACT = 0, 1
LAYOUT_AUTO, LAYOUT_SITE, LAYOUT_REPLICA, LAYOUT_BLOCK = 0, 1, 2, 3
LAUNCH_PLAIN, LAUNCH_PERSISTENT, LAUNCH_GRAPH, LAUNCH_AUTO = 0, 1, 2, 3
INIT_GIVEN, INIT_COLD_Z, INIT_RANDOM = 0, 1, 2
(POLICY_RANDOM, POLICY_FLIP, POLICY_SMALL_STEP, POLICY_GAUSSIAN, POLICY_HN,
 POLICY_ADAPTIVE) = range(6)
SIGMA_MIN, SIGMA_MAX = 1e-4, 60.0
THERMAL_FIELDS = ("e", "m_abs", "m2", "m4", "cv", "chi", "u4", "v1", "v2")
RUN_TRACE_ACCEPTS = 0x1
RUN_DEBUG_NAN_FIELD, RUN_DEBUG_WAIT_CAP = 0x2, 0x4
LAYOUT_NAMES = {1: "site", 2: "replica", 3: "block"}

STATUS = {0: "HSIM_OK", -1: "HSIM_E_ARG", -2: "HSIM_E_CSR", -3: "HSIM_E_PARAM",
          -4: "HSIM_E_STATE", -5: "HSIM_E_DEVICE", -6: "HSIM_E_UNSUPPORTED",
          -7: "HSIM_E_TIMEOUT", -8: "HSIM_E_NUMERIC"}


class HsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_bonds", ctypes.c_int64),
                ("n_colours", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("colour_size", ctypes.c_int64 * 64), ("mean_degree", ctypes.c_double),
                ("uniform_anisotropy", ctypes.c_int32), ("uniform_field_dir", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("n_rep", ctypes.c_int32),
                ("n_phases", ctypes.c_int32), ("total_sites", ctypes.c_int64),
                ("lds_resident", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sites_per_wave", ctypes.c_int32), ("masked_store", ctypes.c_int32),
                ("tuned_launch", ctypes.c_int32), ("persistent_grid", ctypes.c_int32)]


_lib = None
_vp, _i32, _i64, _u32, _u64, _dbl, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_size_t)
_SIGNATURES = {
    "hsim_plan_create": [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _u32],
    "hsim_plan_info": [_vp, _vp],
    "hsim_plan_colouring": [_vp, _vp],
    "hsim_plan_bonds": [_vp, _vp, _vp],
    "hsim_plan_half_rows": [_vp, _vp, _vp, _vp],
    "hsim_batch_create": [_vp, _i32, _vp, _u64, _vp, _i32, _i32],
    "hsim_batch_info": [_vp, _vp],
    "hsim_batch_set_shape": [_vp, _i32, _i32],
    "hsim_batch_set_order": [_vp, _i32],
    "hsim_batch_sizes": [_vp, _i32, _i32, _vp, _vp, _vp],
    "hsim_batch_bind": [_vp, _i32, _i32, _vp, _vp, _vp],
    "hsim_batch_init_spins": [_vp, _i32, _vp, _vp],
    "hsim_batch_run": [_vp, _i32, _i32, _vp, _vp, _i32, _i32, _u32, _vp, _vp],
    "hsim_batch_spins_to_user": [_vp, _i32, _vp, _vp],
    "hsim_batch_status": [_vp, _vp],
    "hsim_autotune": [_vp, ctypes.c_char_p, _i32, _vp],
    "hsim_choose_layout": [_i32, _vp, _u64, _vp, _i32, _vp, _vp, _i32, _vp, _vp],
    "hsim_batch_time_phases": [_vp, _i32],
    "hsim_plan_set_types": [_vp, _vp],
    "hsim_plan_set_site_terms": [_vp, _vp, _vp],
    "hsim_batch_set_policies": [_vp, _i32, _vp, _vp, _dbl, _dbl],
    "hsim_batch_sigma": [_vp, _vp],
    "hsim_batch_bind_outputs": [_vp, _i32, _vp, _vp],
    "hsim_batch_phase_times": [_vp, _vp, _vp, _vp],
    "hsim_energy_prepare": [_vp],
    "hsim_energy_forward_noalloc": [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _vp],
    "hsim_energy_forward": [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _vp],
    "hsim_energy_backward": [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp],
    "hsim_fluct_estimate": [_i64, _dbl, _vp, _vp, _vp, _vp, _vp],
    "hsim_fluct_weights": [_i64, _dbl, _vp, _dbl, _vp, _vp],
    "hsim_spins_planar": [_i64, _i64, _vp, _i32, _vp, _vp],
    "hsim_analysis_thermal": [_vp, _i32, _i32, _i32, _i32, _i64, _vp, _i32, _vp, _vp, _vp],
    "hsim_analysis_tau": [_vp, _i32, _i32, _i32, _i32, _i32, _dbl, _vp, _vp, _vp],
    "hsim_analysis_multihist": [_vp, _i32, _i32, _i32, _i32, _i64, _i32, _vp, _vp, _i32, _vp,
                                _i32, _dbl, _vp, _vp, _vp, _vp],
}
EXPORTED = sorted(list(_SIGNATURES) + ["hsim_plan_destroy", "hsim_batch_destroy",
                                       "hsim_last_error", "hsim_version"])


def lib():
    """Load libhsim.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int32
        L.hsim_plan_destroy.argtypes = [_vp]
        L.hsim_plan_destroy.restype = None
        L.hsim_batch_destroy.argtypes = [_vp]
        L.hsim_batch_destroy.restype = None
        L.hsim_last_error.restype = ctypes.c_char_p
        L.hsim_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise HsimError(code, lib().hsim_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


def _stream():
    """The current torch stream (None, the null stream, when no GPU is
    visible: then only host-side argument checks can run)."""
    if not torch.cuda.is_available():
        return None
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------ thin wrappers
def hsim_plan_create(n, row_ptr, col, J, k=None, axis=None, field_dir=None):
    out = ctypes.c_void_p()
    _check(lib().hsim_plan_create(ctypes.byref(out), n, _ptr(row_ptr), _ptr(col), _ptr(J),
                                  _ptr(k), _ptr(axis), _ptr(field_dir), 0))
    return out


def hsim_plan_info(plan):
    info = PlanInfo()
    _check(lib().hsim_plan_info(plan, ctypes.byref(info)))
    return info


def hsim_plan_colouring(plan, n):
    c = np.empty(max(n, 1), dtype=np.int32)
    _check(lib().hsim_plan_colouring(plan, _ptr(c)))
    return c[:n]


def hsim_plan_bonds(plan):
    nb = ctypes.c_int64()
    _check(lib().hsim_plan_bonds(plan, None, ctypes.byref(nb)))
    ij = np.empty(2 * max(nb.value, 1), dtype=np.int32)
    _check(lib().hsim_plan_bonds(plan, _ptr(ij), None))
    return ij[:2 * nb.value].reshape(nb.value, 2)


def hsim_plan_half_rows(plan, n):
    """(col, bond) [width][n] of the energy forward's half rows."""
    w = ctypes.c_int32()
    _check(lib().hsim_plan_half_rows(plan, ctypes.byref(w), None, None))
    col = np.empty((w.value, n), dtype=np.int32)
    bond = np.empty((w.value, n), dtype=np.int32)
    if col.size:
        _check(lib().hsim_plan_half_rows(plan, None, _ptr(col), _ptr(bond)))
    return col, bond


def hsim_plan_set_types(plan, site_type):
    t = None if site_type is None else np.ascontiguousarray(site_type, dtype=np.int32)
    _check(lib().hsim_plan_set_types(plan, _ptr(t)))


def hsim_plan_set_site_terms(plan, k_cubic=None, spin_norm=None):
    kc = None if k_cubic is None else np.ascontiguousarray(k_cubic, dtype=np.float64)
    mu = None if spin_norm is None else np.ascontiguousarray(spin_norm, dtype=np.float64)
    _check(lib().hsim_plan_set_site_terms(plan, _ptr(kc), _ptr(mu)))


def hsim_plan_destroy(plan):
    lib().hsim_plan_destroy(plan)


def hsim_batch_create(plans, seed, replica_ids=None, precision=FP32, layout=LAYOUT_AUTO):
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    ids = None if replica_ids is None else np.ascontiguousarray(replica_ids, dtype=np.uint32)
    out = ctypes.c_void_p()
    _check(lib().hsim_batch_create(ctypes.byref(out), len(plans), arr, seed & (2 ** 64 - 1),
                                   _ptr(ids), precision, layout))
    return out


def hsim_batch_info(batch):
    info = BatchInfo()
    _check(lib().hsim_batch_info(batch, ctypes.byref(info)))
    return info


def hsim_batch_set_shape(batch, sites_per_wave, masked_store):
    _check(lib().hsim_batch_set_shape(batch, sites_per_wave, masked_store))


def hsim_batch_set_order(batch, plane_sites):
    _check(lib().hsim_batch_set_order(batch, plane_sites))


def hsim_batch_sizes(batch, n_steps, mcs):
    ws, sp, hi = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().hsim_batch_sizes(batch, n_steps, mcs, ctypes.byref(ws), ctypes.byref(sp),
                                  ctypes.byref(hi)))
    return ws.value, sp.value, hi.value


def hsim_batch_bind(batch, n_steps, mcs, ws, spins, history):
    _check(lib().hsim_batch_bind(batch, n_steps, mcs, _ptr(ws), _ptr(spins), _ptr(history)))


def hsim_batch_init_spins(batch, mode, host_spins=None):
    hs = None if host_spins is None else np.ascontiguousarray(host_spins, dtype=np.float64)
    _check(lib().hsim_batch_init_spins(batch, mode, _ptr(hs), _stream()))


def hsim_batch_run(batch, first_step, T, B, recompute_every=100, launch=LAUNCH_AUTO,
                   trace=None, debug_flags=0):
    T = np.ascontiguousarray(T, dtype=np.float64)
    B = np.ascontiguousarray(np.broadcast_to(B, T.shape), dtype=np.float64)
    n_steps = T.shape[-1]
    flags = (RUN_TRACE_ACCEPTS if trace is not None else 0) | debug_flags
    _check(lib().hsim_batch_run(batch, first_step, n_steps, _ptr(T), _ptr(B), recompute_every,
                                launch, flags, _ptr(trace), _stream()))


def hsim_batch_spins_to_user(batch, rep, out):
    _check(lib().hsim_batch_spins_to_user(batch, rep, _ptr(out), _stream()))


def hsim_batch_status(batch):
    s = ctypes.c_int32()
    _check(lib().hsim_batch_status(batch, ctypes.byref(s)))
    return s.value


def hsim_autotune(batch, cache_path=None, trial_mcs=20):
    cp = None if cache_path is None else cache_path.encode()
    _check(lib().hsim_autotune(batch, cp, trial_mcs, _stream()))


def hsim_choose_layout(plans, seed, T, B, replica_ids=None, precision=FP32, trial_mcs=10):
    """plans: Plan handles; T, B: one temperature and field per replica."""
    arr = (ctypes.c_void_p * len(plans))(*[p.value for p in plans])
    ids = None if replica_ids is None else np.ascontiguousarray(replica_ids, dtype=np.uint32)
    Tv = np.ascontiguousarray(np.broadcast_to(np.asarray(T, dtype=np.float64), (len(plans),)))
    Bv = np.ascontiguousarray(np.broadcast_to(np.asarray(B, dtype=np.float64), (len(plans),)))
    out = ctypes.c_int32(-1)
    _check(lib().hsim_choose_layout(len(plans), arr, seed & (2 ** 64 - 1), _ptr(ids), precision,
                                    _ptr(Tv), _ptr(Bv), trial_mcs, ctypes.byref(out), _stream()))
    return out.value


def hsim_batch_set_policies(batch, policies, sigma_min=SIGMA_MIN, sigma_max=SIGMA_MAX):
    pol = np.ascontiguousarray([int(a) for a, _ in policies], dtype=np.int32)
    prm = np.ascontiguousarray([float(b) for _, b in policies], dtype=np.float64)
    _check(lib().hsim_batch_set_policies(batch, len(policies), _ptr(pol) if len(pol) else None,
                                         _ptr(prm) if len(prm) else None, float(sigma_min),
                                         float(sigma_max)))


def hsim_batch_bind_outputs(batch, n_types, type_mag, snapshots):
    _check(lib().hsim_batch_bind_outputs(batch, n_types, _ptr(type_mag), _ptr(snapshots)))


def hsim_batch_sigma(batch, n_rep):
    out = np.empty(n_rep)
    _check(lib().hsim_batch_sigma(batch, _ptr(out)))
    return out


def hsim_batch_time_phases(batch, every):
    _check(lib().hsim_batch_time_phases(batch, every))


def hsim_batch_phase_times(batch):
    ms, n, u = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().hsim_batch_phase_times(batch, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
    return ms.value, n.value, u.value


def hsim_batch_destroy(batch):
    lib().hsim_batch_destroy(batch)


def hsim_energy_prepare(plan):
    _check(lib().hsim_energy_prepare(plan))


def hsim_energy_forward(plan, batch, precision, spins, J_bond, k, axis, B, field_dir, E):
    _check(lib().hsim_energy_forward(plan, batch, precision, _ptr(spins), _ptr(J_bond), _ptr(k),
                                     _ptr(axis), float(B), _ptr(field_dir), _ptr(E), _stream()))


def hsim_energy_forward_noalloc(plan, batch, precision, spins, J_bond, k, axis, B, field_dir, E):
    _check(lib().hsim_energy_forward_noalloc(plan, batch, precision, _ptr(spins), _ptr(J_bond),
                                             _ptr(k), _ptr(axis), float(B), _ptr(field_dir),
                                             _ptr(E), _stream()))


def hsim_energy_backward(plan, batch, precision, spins, J_bond, k, axis, B, field_dir, gE,
                         gS=None, gJ=None, gk=None, gB=None):
    _check(lib().hsim_energy_backward(plan, batch, precision, _ptr(spins), _ptr(J_bond), _ptr(k),
                                      _ptr(axis), float(B), _ptr(field_dir), _ptr(gE), _ptr(gS),
                                      _ptr(gJ), _ptr(gk), _ptr(gB), _stream()))


def hsim_fluct_estimate(n, beta, O, dE, dO, out):
    _check(lib().hsim_fluct_estimate(n, float(beta), _ptr(O), _ptr(dE), _ptr(dO), _ptr(out),
                                     _stream()))


def hsim_fluct_weights(n, beta, O, c, w):
    _check(lib().hsim_fluct_weights(n, float(beta), _ptr(O), float(c), _ptr(w), _stream()))


def hsim_spins_planar(n_cfg, n_sites, spins_in, precision, out):
    _check(lib().hsim_spins_planar(n_cfg, n_sites, _ptr(spins_in), precision, _ptr(out),
                                   _stream()))


def hsim_version():
    return lib().hsim_version().decode()


# ------------------------------------------------------------- objects
def _hist_shape(history):
    if history.dim() != 4 or history.shape[-1] != 5 or history.dtype != torch.float64:
        raise ValueError("history must be a float64 tensor [R][S][M][5]")
    return [int(v) for v in history.shape[:3]]


def hsim_analysis_thermal(history, m0, n_sites, beta, beta_eval=None):
    """Thermal summaries [R][S][n_eval][9] (THERMAL_FIELDS) of every series,
    at the sampling beta [R][S] or reweighted to beta_eval [R][S][n_eval]."""
    R, S, M = _hist_shape(history)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (R, S)))
    be = None if beta_eval is None else np.ascontiguousarray(beta_eval, dtype=np.float64).reshape(R, S, -1)
    ne = 1 if be is None else be.shape[-1]
    out = torch.empty((R, S, ne, 9), dtype=torch.float64, device=history.device)
    _check(lib().hsim_analysis_thermal(_ptr(history), R, S, M, m0, n_sites, _ptr(b), ne, _ptr(be),
                                       _ptr(out), _stream()))
    return out


def hsim_analysis_tau(history, m0, observable=0, c=6.0):
    """Integrated autocorrelation times [R][S] of E (0) or |M| (1), and windows."""
    R, S, M = _hist_shape(history)
    tau = torch.empty((R, S), dtype=torch.float64, device=history.device)
    win = torch.empty((R, S), dtype=torch.int32, device=history.device)
    _check(lib().hsim_analysis_tau(_ptr(history), R, S, M, m0, observable, float(c), _ptr(tau),
                                   _ptr(win), _stream()))
    return tau, win


def hsim_analysis_multihist(history, m0, n_sites, series, beta_k, beta_eval, max_iter=5000,
                            tol=1e-11):
    """Multiple-histogram free energies f [K] (f_0 = 0), iterations, and the
    thermal summaries [n_eval][9] at beta_eval."""
    R, S, M = _hist_shape(history)
    sr = np.ascontiguousarray(series, dtype=np.int32).reshape(-1, 2)
    K = sr.shape[0]
    bk = np.ascontiguousarray(beta_k, dtype=np.float64)
    be = np.ascontiguousarray(np.atleast_1d(beta_eval), dtype=np.float64)
    f = np.empty(K)
    it = ctypes.c_int32()
    out = torch.empty((be.size, 9), dtype=torch.float64, device=history.device)
    _check(lib().hsim_analysis_multihist(_ptr(history), R, S, M, m0, n_sites, K, _ptr(sr), _ptr(bk),
                                         be.size, _ptr(be), max_iter, float(tol), _ptr(f),
                                         ctypes.byref(it), _ptr(out), _stream()))
    return f, it.value, out


class Plan:
    """One lattice: CSR neighbours with per-entry J, per-site k/axis/field
    direction (host arrays; copied by the library)."""

    def __init__(self, lat):
        self.n = int(lat.n)
        self._keep = dict(
            row_ptr=np.ascontiguousarray(lat.row_ptr, dtype=np.int64),
            col=np.ascontiguousarray(lat.col, dtype=np.int32),
            J=np.ascontiguousarray(lat.J, dtype=np.float64),
            k=None if lat.k is None else np.ascontiguousarray(lat.k, dtype=np.float64),
            axis=None if lat.axis is None else np.ascontiguousarray(lat.axis, dtype=np.float64),
            ndir=None if lat.ndir is None else np.ascontiguousarray(lat.ndir, dtype=np.float64))
        kp = self._keep
        self.handle = hsim_plan_create(self.n, kp["row_ptr"], kp["col"], kp["J"], kp["k"],
                                       kp["axis"], kp["ndir"])
        kc, mu = getattr(lat, "kc", None), getattr(lat, "norm", None)
        if kc is not None or mu is not None:
            hsim_plan_set_site_terms(self.handle, kc, mu)
        self.info = hsim_plan_info(self.handle)

    def colouring(self):
        return hsim_plan_colouring(self.handle, self.n)

    def bonds(self):
        return hsim_plan_bonds(self.handle)

    def half_rows(self):
        return hsim_plan_half_rows(self.handle, self.n)

    def set_types(self, site_type):
        """Site types (user order, 0..7), or None for type 0 everywhere."""
        hsim_plan_set_types(self.handle, site_type)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            hsim_plan_destroy(h)
            self.handle = None


class Batch:
    """Replicas over plans with caller-owned (torch) device buffers."""

    @staticmethod
    def choose_layout(plans, seed, T, B, replica_ids=None, precision=FP32, trial_mcs=10):
        """The layout to create the batch with, chosen by timing (hsim_choose_layout)."""
        return hsim_choose_layout([p.handle for p in plans], seed, T, B, replica_ids, precision,
                                  trial_mcs)

    def __init__(self, plans, seed, replica_ids=None, precision=FP32, layout=LAYOUT_AUTO,
                 device="cuda"):
        self.plans = list(plans)
        self.R = len(self.plans)
        self.precision = precision
        self.handle = hsim_batch_create([p.handle for p in self.plans], seed, replica_ids,
                                        precision, layout)
        self.info = hsim_batch_info(self.handle)
        self.device = device
        self.ws = self.spins = self.history = None

    @property
    def layout(self):
        return LAYOUT_NAMES[self.info.layout]

    def bind(self, n_steps, mcs):
        ws, sp, hi = hsim_batch_sizes(self.handle, n_steps, mcs)
        self.n_steps, self.mcs = n_steps, mcs
        self.ws = torch.zeros(ws, dtype=torch.uint8, device=self.device)
        self.spins = torch.zeros(sp, dtype=torch.uint8, device=self.device)
        self.history = torch.zeros((self.R, n_steps, mcs, 5), dtype=torch.float64,
                                   device=self.device)
        hsim_batch_bind(self.handle, n_steps, mcs, self.ws, self.spins, self.history)
        return self

    def init_spins(self, mode, host_spins=None):
        hsim_batch_init_spins(self.handle, mode, host_spins)

    def run(self, T, B, first_step=0, recompute_every=100, launch=LAUNCH_AUTO, trace=None,
            debug_flags=0):
        T = np.asarray(T, dtype=np.float64)
        if T.ndim == 1:
            T = np.broadcast_to(T, (self.R, T.size))
        B = np.broadcast_to(np.asarray(B, dtype=np.float64), T.shape)
        hsim_batch_run(self.handle, first_step, T, B, recompute_every, launch, trace, debug_flags)

    def new_trace(self, n_steps_run):
        words = (max(p.n for p in self.plans) + 31) // 32
        return torch.zeros((self.R, n_steps_run * self.mcs, words), dtype=torch.int32,
                           device=self.device)

    def spins_user(self, rep):
        out = torch.empty((self.plans[rep].n, 3), dtype=torch.float64, device=self.device)
        hsim_batch_spins_to_user(self.handle, rep, out)
        return out

    def status(self):
        torch.cuda.current_stream().synchronize()
        return hsim_batch_status(self.handle)

    def autotune(self, cache_path=None, trial_mcs=20):
        hsim_autotune(self.handle, cache_path, trial_mcs)
        self.info = hsim_batch_info(self.handle)

    def set_shape(self, sites_per_wave, masked_store=0):
        """Replica layout: tile shape and store policy (the tuner's knobs)."""
        hsim_batch_set_shape(self.handle, sites_per_wave, masked_store)
        self.info = hsim_batch_info(self.handle)

    def set_order(self, plane_sites):
        """Replica layout: dispatch order of the tiles (-1 derived, 0 in order,
        > 1 plane stride in sites of a class); changes no result."""
        hsim_batch_set_order(self.handle, plane_sites)

    def set_policies(self, policies, sigma_min=SIGMA_MIN, sigma_max=SIGMA_MAX):
        """policies: list of (POLICY_*, param) per site type; [] for the
        random move everywhere."""
        hsim_batch_set_policies(self.handle, policies, sigma_min, sigma_max)
        return self

    def bind_outputs(self, type_mag_types=0, snapshots=False):
        """Allocate and attach the optional outputs: self.type_mag
        [R][S][M][n_types][3] (type_mag_types > 0) and self.snapshots
        [R][S][n_max][3] (snapshots=True); 0 / False detaches."""
        S, M = self.n_steps, self.mcs
        nmax = max(p.n for p in self.plans)
        self.type_mag = (torch.zeros((self.R, S, M, type_mag_types, 3), dtype=torch.float64,
                                     device=self.device) if type_mag_types > 0 else None)
        self.snapshots = (torch.zeros((self.R, S, nmax, 3), dtype=torch.float64, device=self.device)
                          if snapshots else None)
        hsim_batch_bind_outputs(self.handle, type_mag_types, self.type_mag, self.snapshots)
        return self

    def sigma(self):
        """Current adaptive width of every replica (host array)."""
        torch.cuda.current_stream().synchronize()
        return hsim_batch_sigma(self.handle, self.R)

    def time_phases(self, every):
        hsim_batch_time_phases(self.handle, every)

    def phase_times(self):
        """(total ms, timed launches, updates of those launches)."""
        return hsim_batch_phase_times(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            hsim_batch_destroy(h)
            self.handle = None


def unpack_trace(trace, n):
    """Bitmap [.., words] (int32) -> bool array [.., n]."""
    t = trace.cpu().numpy().view(np.uint32)
    bits = (t[..., :, None] >> np.arange(32, dtype=np.uint32)) & 1
    return bits.reshape(*t.shape[:-1], -1)[..., :n].astype(bool)
