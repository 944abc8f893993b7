"""CPU oracle of the Heisenberg Metropolis hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it to check and time the GPU library.
It never imports the GPU package and the GPU package never imports it.

The C source (``hsim_oracle.c``) is plain serial double precision; this module
builds it with gcc on first use (``build()``), marshals numpy arrays, and adds
nothing to the arithmetic.  Citations refer to the paper's sections:
  * Eq. 1-2 ("Classical spin Hamiltonian"): the energy, one term per bond.
  * Eq. 4 and the MCS definition ("Monte Carlo Metropolis algorithm").
  * the stored history of energy and magnetisation at every MCS of every
    temperature/field step ("VEGAS software package").
"""
import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

PROPOSAL_EXACT, PROPOSAL_F32MAP = 0, 1
# update policies (the moves of Hinzke and Nowak 1999 named in the paper's
# "Monte Carlo Metropolis algorithm" section, and the adaptive move)
POLICY_RANDOM, POLICY_FLIP, POLICY_SMALL_STEP, POLICY_GAUSSIAN, POLICY_HN, POLICY_ADAPTIVE = range(6)
SIGMA_MIN, SIGMA_MAX = 1e-4, 60.0
INIT_GIVEN, INIT_COLD_Z, INIT_RANDOM = 0, 1, 2
INIT_CODES = {"given": INIT_GIVEN, "cold": INIT_COLD_Z, "random": INIT_RANDOM}


def build(force=True):
    """Compile the oracle into liboracle.so (gcc, -O2, no FP contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Lattice(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("J", ctypes.c_void_p), ("k", ctypes.c_void_p), ("axis", ctypes.c_void_p),
                ("ndir", ctypes.c_void_p), ("kc", ctypes.c_void_p), ("norm", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("replica", ctypes.c_uint32),
                ("n_steps", ctypes.c_int32), ("mcs_per_step", ctypes.c_int32),
                ("first_step", ctypes.c_int32), ("recompute_every", ctypes.c_int32),
                ("T", ctypes.c_void_p), ("B", ctypes.c_void_p), ("proposal", ctypes.c_int32),
                ("init", ctypes.c_int32), ("order", ctypes.c_void_p), ("colour", ctypes.c_void_p),
                ("check_every_update", ctypes.c_int32),
                ("n_types", ctypes.c_int32), ("site_type", ctypes.c_void_p),
                ("type_policy", ctypes.c_void_p), ("type_param", ctypes.c_void_p),
                ("sigma_min", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("sigma", ctypes.c_void_p), ("sigma_trace", ctypes.c_void_p)]


class _Outputs(ctypes.Structure):
    _fields_ = [("spins", ctypes.c_void_p), ("history", ctypes.c_void_p),
                ("accept", ctypes.c_void_p), ("e_full", ctypes.c_void_p),
                ("near_ties", ctypes.c_int64), ("max_incr_err", ctypes.c_double),
                ("max_update_err", ctypes.c_double), ("n_decisions", ctypes.c_int64),
                ("type_mag", ctypes.c_void_p), ("snapshots", ctypes.c_void_p),
                ("dE_trace", ctypes.c_void_p), ("u_trace", ctypes.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
            vp, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double)
            L.or_philox_batch.argtypes = [i64, vp, vp, vp]
            L.or_u53.argtypes = [u32, u32]
            L.or_u53.restype = dbl
            L.or_u24.argtypes = [u32]
            L.or_u24.restype = dbl
            L.or_sphere_exact.argtypes = [u64, u32, u32, u32, vp]
            L.or_sphere_exact.restype = ctypes.c_int
            L.or_sphere_f32map.argtypes = [u64, u32, u32, u32, vp, vp]
            L.or_validate.argtypes = [vp]
            L.or_validate.restype = ctypes.c_int
            L.or_greedy_colour.argtypes = [vp, vp]
            L.or_greedy_colour.restype = ctypes.c_int
            L.or_count_conflicts.argtypes = [vp, vp]
            L.or_count_conflicts.restype = i64
            L.or_energy.argtypes = [vp, dbl, vp, vp, vp, vp, vp]
            L.or_energy.restype = dbl
            L.or_bonds.argtypes = [vp, vp, vp]
            L.or_bonds.restype = i64
            L.or_energy_grad.argtypes = [vp, dbl, vp, dbl, vp, vp, vp, vp]
            L.or_run.argtypes = [vp, vp, vp]
            L.or_run.restype = ctypes.c_int
            L.or_log.argtypes = [dbl]
            L.or_log.restype = dbl
            L.or_trial.argtypes = [ctypes.c_int32, ctypes.c_int32, u64, u32, u32, u32, vp, dbl,
                                   dbl, vp]
            L.or_trial.restype = dbl
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Lat:
    """Keeps contiguous copies alive for the C structure."""

    def __init__(self, lat):
        self.row_ptr = np.ascontiguousarray(lat.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(lat.col, dtype=np.int32)
        self.J = np.ascontiguousarray(lat.J, dtype=np.float64)
        self.k = None if lat.k is None else np.ascontiguousarray(lat.k, dtype=np.float64)
        self.axis = None if lat.axis is None else np.ascontiguousarray(lat.axis, dtype=np.float64)
        self.ndir = None if lat.ndir is None else np.ascontiguousarray(lat.ndir, dtype=np.float64)
        kc, norm = getattr(lat, "kc", None), getattr(lat, "norm", None)
        self.kc = None if kc is None else np.ascontiguousarray(kc, dtype=np.float64)
        self.norm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float64)
        self.n = int(lat.n)
        self.s = _Lattice(self.n, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.J),
                          _ptr(self.k), _ptr(self.axis), _ptr(self.ndir), _ptr(self.kc),
                          _ptr(self.norm))

    @property
    def ref(self):
        return ctypes.byref(self.s)


# --------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 words for counters ctr (m, 4) uint32 and key (2,) uint32."""
    ctr = np.ascontiguousarray(np.atleast_2d(ctr), dtype=np.uint32)
    key = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    lib().or_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def u53(hi, lo):
    return lib().or_u53(int(hi), int(lo))


def u24(w):
    return lib().or_u24(int(w))


def sphere_exact(seed, site, g, rep):
    out = np.empty(3)
    t = lib().or_sphere_exact(seed, site, g, rep, _ptr(out))
    return out, t


def sphere_f32map(seed, site, g, rep):
    out = np.empty(3)
    u = np.empty(1)
    lib().or_sphere_f32map(seed, site, g, rep, _ptr(out), _ptr(u))
    return out, float(u[0])


def log(x):
    """The oracle's own natural logarithm (or_log)."""
    return lib().or_log(float(x))


def trial(proposal, policy, seed, site, g, rep, s, param, cos_theta=None):
    """Trial direction of one site: returns (trial (3,), acceptance uniform)."""
    out = np.empty(3)
    s = np.ascontiguousarray(s, dtype=np.float64)
    c = np.cos(param) if cos_theta is None else cos_theta
    u = lib().or_trial(proposal, policy, seed, site, g, rep, _ptr(s), float(param), float(c),
                       _ptr(out))
    return out, u


def validate(lat):
    L = _Lat(lat)
    return lib().or_validate(L.ref)


def greedy_colour(lat):
    """Greedy colouring in breadth-first order: components by lowest site
    index, each searched breadth-first from that site with neighbours queued
    in CSR order; every site takes the smallest colour no coloured neighbour
    has."""
    L = _Lat(lat)
    c = np.empty(max(lat.n, 1), dtype=np.int32)
    nc = lib().or_greedy_colour(L.ref, _ptr(c))
    return c[:lat.n], nc


def count_conflicts(lat, colour):
    L = _Lat(lat)
    colour = np.ascontiguousarray(colour, dtype=np.int32)
    return lib().or_count_conflicts(L.ref, _ptr(colour))


def energy(lat, B, spins):
    """Eq. 1 for spins (n, 3): returns dict E, ex, zee, ani, scale."""
    L = _Lat(lat)
    S = np.ascontiguousarray(spins, dtype=np.float64).reshape(-1)
    parts = np.zeros(4)
    ex, zee, ani, sc = (ctypes.c_double(), ctypes.c_double(), ctypes.c_double(),
                        ctypes.c_double())
    E = lib().or_energy(L.ref, float(B), _ptr(S), ctypes.addressof(ex), ctypes.addressof(zee),
                        ctypes.addressof(ani), ctypes.addressof(sc))
    del parts
    return dict(E=E, ex=ex.value, zee=zee.value, ani=ani.value, scale=sc.value)


def bonds(lat):
    L = _Lat(lat)
    nb = lib().or_bonds(L.ref, None, None)
    ij = np.empty(2 * max(nb, 1), dtype=np.int32)
    Jb = np.empty(max(nb, 1))
    lib().or_bonds(L.ref, _ptr(ij), _ptr(Jb))
    return ij[:2 * nb].reshape(nb, 2), Jb[:nb]


def energy_grad(lat, B, spins, g=1.0):
    """g * (dE/dS (n,3), dE/dJ_bond (nb,), dE/dk (n,), dE/dB)."""
    L = _Lat(lat)
    S = np.ascontiguousarray(spins, dtype=np.float64).reshape(-1)
    nb = lib().or_bonds(L.ref, None, None)
    gS = np.zeros(3 * lat.n)
    gJ = np.zeros(max(nb, 1))
    gk = np.zeros(max(lat.n, 1))
    gB = ctypes.c_double(0.0)
    lib().or_energy_grad(L.ref, float(B), _ptr(S), float(g), _ptr(gS), _ptr(gJ), _ptr(gk),
                         ctypes.addressof(gB))
    return gS.reshape(lat.n, 3), gJ[:nb], gk[:lat.n], gB.value


def run(lat, T, B, mcs_per_step, seed, replica=0, init="random", spins=None,
        proposal=PROPOSAL_EXACT, first_step=0, recompute_every=100, order=None,
        colour=None, trace_accepts=False, full_energy=False, check_every_update=False,
        policies=None, site_type=None, sigma=None, sigma_min=SIGMA_MIN, sigma_max=SIGMA_MAX,
        trace_sigma=False, type_mag=False, snapshots=False, decision_trace=False):
    """Colour-ordered Metropolis sweep of one replica over a T/B schedule.

    policies: None (random move everywhere) or a list of (policy, param) per
    site type; site_type: per-site type in user order (None: type 0); sigma:
    starting adaptive width (default: the adaptive type's param).
    type_mag: record the magnetisation of every site type after every MCS
    (site types from site_type, as many types as policies; without policies
    one type); snapshots: record the spins at the end of every step.

    Returns a dict: history (S, M, 5) [E, Mx, My, Mz, n_acc], spins (n, 3),
    accept (S*M, n) uint8 or None, e_full (S*M,) or None, near_ties,
    max_incr_err, max_update_err, n_decisions, sigma (final adaptive width or
    None), sigma_trace ((S*M,) width used in each MCS, or None), type_mag
    ((S, M, n_types, 3) or None), snapshots ((S, n, 3) or None).
    """
    T = np.ascontiguousarray(np.atleast_1d(T), dtype=np.float64)
    B = np.ascontiguousarray(np.broadcast_to(np.atleast_1d(B), T.shape), dtype=np.float64)
    S_steps, M, n = T.size, int(mcs_per_step), int(lat.n)
    L = _Lat(lat)
    if spins is None:
        spins = np.zeros((n, 3))
        if init == "given":
            raise ValueError("init='given' needs spins")
    sp = np.ascontiguousarray(spins, dtype=np.float64).reshape(n, 3).copy()
    hist = np.zeros((S_steps, M, 5))
    acc = np.zeros((S_steps * M, n), dtype=np.uint8) if trace_accepts else None
    ef = np.zeros(S_steps * M) if full_energy else None
    order_a = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
    colour_a = None if colour is None else np.ascontiguousarray(colour, dtype=np.int32)
    ntypes, tp, tq, st, sg, strace = 0, None, None, None, None, None
    if policies is not None:
        ntypes = len(policies)
        tp = np.ascontiguousarray([int(a) for a, _ in policies], dtype=np.int32)
        tq = np.ascontiguousarray([float(b) for _, b in policies], dtype=np.float64)
        if site_type is not None:
            st = np.ascontiguousarray(site_type, dtype=np.int32)
        ad = [b for a, b in policies if int(a) == POLICY_ADAPTIVE]
        sg = np.array([float(sigma) if sigma is not None else (ad[0] if ad else 1.0)])
        if trace_sigma:
            strace = np.zeros(S_steps * M)
    p = _Params(seed & 0xFFFFFFFFFFFFFFFF, replica, S_steps, M, first_step, recompute_every,
                _ptr(T), _ptr(B), proposal, INIT_CODES[init] if isinstance(init, str) else init,
                _ptr(order_a), _ptr(colour_a), 1 if check_every_update else 0,
                ntypes, _ptr(st), _ptr(tp), _ptr(tq), float(sigma_min), float(sigma_max),
                _ptr(sg), _ptr(strace))
    nt = max(ntypes, 1)
    tm = np.zeros((S_steps, M, nt, 3)) if type_mag else None
    snap = np.zeros((S_steps, n, 3)) if snapshots else None
    dtr = np.zeros((S_steps * M, n)) if decision_trace else None
    utr = np.zeros((S_steps * M, n)) if decision_trace else None
    o = _Outputs(_ptr(sp), _ptr(hist), _ptr(acc), _ptr(ef), 0, 0.0, 0.0, 0, _ptr(tm), _ptr(snap),
                 _ptr(dtr), _ptr(utr))
    rc = lib().or_run(L.ref, ctypes.byref(p), ctypes.byref(o))
    if rc != 0:
        raise ValueError(f"oracle run rejected its input (code {rc})")
    has_ad = policies is not None and any(int(a) == POLICY_ADAPTIVE for a, _ in policies)
    return dict(history=hist, spins=sp, accept=acc, e_full=ef, near_ties=o.near_ties,
                max_incr_err=o.max_incr_err, max_update_err=o.max_update_err,
                n_decisions=o.n_decisions, sigma=float(sg[0]) if has_ad else None,
                sigma_trace=strace, type_mag=tm, snapshots=snap, dE_trace=dtr, u_trace=utr)


def run_replicas(jobs, threads=None):
    """Run independent replicas in a thread pool (one replica per thread; the
    C call releases the GIL).  jobs: list of dicts of ``run`` arguments.
    Returns (results, threads_used)."""
    threads = threads or os.cpu_count() or 1
    threads = max(1, min(threads, len(jobs)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda kw: run(**kw), jobs))
    return res, threads


def fluct_gradients(lat, B, spins, beta, O=None):
    """Fluctuation estimate of the derivatives of a canonical average with
    respect to every per-bond exchange constant, every anisotropy constant and
    the field intensity, from configurations sampled at inverse temperature
    beta.  Differentiating the Boltzmann average of Eq. 4's stationary
    distribution (section "Thermal averages": responses as fluctuations):

        d<O>/dtheta = <dO/dtheta> - beta (<O dE/dtheta> - <O><dE/dtheta>)

    spins: (n_cfg, n, 3); O: per-configuration observable that does not
    depend on the parameters (None: O = E itself, whose own derivative is
    dE/dtheta).  dE/dtheta of every configuration comes from energy_grad.
    Returns dict gJ (n_bonds,), gk (n,), gB (scalar): plain sample means."""
    spins = np.asarray(spins, dtype=np.float64)
    nc = spins.shape[0]
    dJ, dk, dB, Es = [], [], [], []
    for s in spins:
        _, gJ, gk, gB = energy_grad(lat, B, s)
        dJ.append(gJ)
        dk.append(gk)
        dB.append(gB)
        Es.append(energy(lat, B, s)["E"])
    dJ, dk, dB = np.array(dJ), np.array(dk), np.array(dB)
    own = O is None
    O = np.array(Es) if own else np.asarray(O, dtype=np.float64).reshape(nc)
    dO = O - O.mean()

    def est(X):
        cov = np.tensordot(dO, X - X.mean(axis=0), axes=(0, 0)) / nc
        return (X.mean(axis=0) if own else 0.0) - beta * cov

    return dict(gJ=est(dJ), gk=est(dk), gB=float(est(dB)), O=O)
