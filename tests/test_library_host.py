"""Host-side checks of libhsim.so that need no GPU: the library loads and
exports every entry point include/hsim.h declares; lattice ingest validates
its input and its colouring and bond order equal the oracle's (independent
implementations of the same rule: bit-exact integer parity); batch layout
choice, sizes and call-order errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1803_07030_amd import hsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "hsim.h")).read()
    body = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(hsim_[a-z_]+)\s*\(", body))
    assert "hsim_batch_run" in declared and len(declared) >= 20
    L = hsim.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(hsim.EXPORTED) == declared
    assert hsim.hsim_version().startswith("hsim")


def _lat_variants():
    return [synth.sc_periodic(8), synth.sc_periodic(5, 5, 3), synth.core_shell_ball(R=10, Rc=7),
            synth.diluted_film(19, 4, seed=11), synth.random_tree(300, seed=5),
            synth.open_chain(17), synth.isolated(10),
            synth.from_bonds(5, *np.triu_indices(5, 1), np.ones(10))]


@pytest.mark.parametrize("idx", range(8))
def test_colouring_and_bonds_equal_oracle(idx):
    lat = _lat_variants()[idx]
    p = hsim.Plan(lat)
    c_ref, nc = oracle.greedy_colour(lat)
    assert np.array_equal(p.colouring(), c_ref)
    assert p.info.n_colours == nc
    assert list(p.info.colour_size[:nc]) == list(np.bincount(c_ref, minlength=nc))
    b_ref, _ = oracle.bonds(lat)
    assert np.array_equal(p.bonds(), b_ref)
    assert p.info.n_bonds == lat.n_bonds


def _random_graph(n, maxd, seed):
    rng = np.random.default_rng(seed)
    deg = np.zeros(n, dtype=np.int64)
    pairs = set()
    for _ in range(6 * n):
        a, b = (int(x) for x in rng.integers(0, n, 2))
        if a == b or deg[a] >= maxd or deg[b] >= maxd or (min(a, b), max(a, b)) in pairs:
            continue
        pairs.add((min(a, b), max(a, b)))
        deg[a] += 1
        deg[b] += 1
    bi, bj = (np.array(x) for x in zip(*sorted(pairs)))
    return synth.from_bonds(n, bi, bj, np.ones(bi.size))


@pytest.mark.parametrize("idx", range(11))
def test_half_rows_hold_every_bond_once(idx):
    """The energy forward's half rows (each bond at the end a closed-walk
    orientation makes it leave): every bond exactly once, its far end and
    bond id as the lattice has them, at most ceil(d/2) bonds per site of
    degree d, empty slots naming the site itself; no half rows when a site's
    degree exceeds 8."""
    lats = _lat_variants() + [_random_graph(500, 8, 1), _random_graph(701, 7, 2),
                              synth.sc_periodic(3)]
    lat = lats[idx]
    p = hsim.Plan(lat)
    col, bond = p.half_rows()
    deg = np.diff(lat.row_ptr)
    if deg.max(initial=0) > 8:
        assert col.shape[0] == 0
        return
    assert col.shape == (3 if deg.max(initial=0) <= 6 else 4, lat.n)
    ij = p.bonds()
    seen = np.zeros(len(ij), dtype=np.int64)
    held = np.zeros(lat.n, dtype=np.int64)
    for q in range(col.shape[0]):
        for i in range(lat.n):
            b, c = bond[q, i], col[q, i]
            if b < 0:
                assert c == i
                continue
            seen[b] += 1
            held[i] += 1
            assert sorted((i, c)) == sorted(ij[b].tolist())
    assert np.all(seen == 1)
    assert np.all(held <= (deg + 1) // 2)


def _expect(code, fn):
    with pytest.raises(hsim.HsimError) as e:
        fn()
    assert e.value.code == code, str(e.value)


def _copy(lat, **kw):
    d = dict(n=lat.n, row_ptr=lat.row_ptr.copy(), col=lat.col.copy(), J=lat.J.copy(), k=lat.k,
             axis=lat.axis, ndir=lat.ndir)
    d.update(kw)
    return synth.Lattice(**d)


def test_plan_rejects_invalid_lattices():
    lat = synth.sc_periodic(4)
    bad = _copy(lat)
    bad.J[3] = 1.5
    _expect(-3, lambda: hsim.Plan(bad))
    bad = _copy(lat)
    bad.col[0] = 0
    _expect(-2, lambda: hsim.Plan(bad))
    bad = _copy(lat)
    bad.col[1] = bad.col[0]
    _expect(-2, lambda: hsim.Plan(bad))
    bad = _copy(lat)
    bad.col[0] = lat.n + 5
    _expect(-2, lambda: hsim.Plan(bad))
    bad = _copy(lat)
    bad.row_ptr[0] = 1
    _expect(-2, lambda: hsim.Plan(bad))
    _expect(-3, lambda: hsim.Plan(_copy(lat, k=np.full(lat.n, np.inf))))
    _expect(-3, lambda: hsim.Plan(_copy(lat, axis=np.tile([0.0, 0.6, 0.6], (lat.n, 1)))))
    _expect(-3, lambda: hsim.Plan(_copy(lat, ndir=np.tile([0.0, 0.0, 2.0], (lat.n, 1)))))
    # a one-way link (missing reverse entry)
    one_way = synth.Lattice(3, np.array([0, 1, 1, 1]), np.array([1], dtype=np.int32),
                            np.array([1.0]))
    _expect(-2, lambda: hsim.Plan(one_way))
    _expect(-1, lambda: hsim.hsim_plan_create(-1, lat.row_ptr, lat.col, lat.J))


def test_plan_flags_uniform_parameters():
    lat = synth.sc_periodic(4)
    assert hsim.Plan(lat).info.uniform_anisotropy == 1
    lat.k = synth.uniform01(1, lat.n)
    assert hsim.Plan(lat).info.uniform_anisotropy == 0
    lat.ndir = synth.unit_vectors(2, lat.n)
    assert hsim.Plan(lat).info.uniform_field_dir == 0


def test_batch_layouts_sizes_and_errors():
    sc = hsim.Plan(synth.sc_periodic(8))
    big = hsim.Plan(synth.sc_periodic(64))
    b = hsim.Batch([sc], seed=0, precision=hsim.FP64_EXACT)
    assert b.layout == "block" and b.info.lds_resident == 1
    ws, sp, hi = hsim.hsim_batch_sizes(b.handle, 20, 1000)
    assert sp == 3 * 512 * 8 and hi == 20 * 1000 * 5 * 8
    b = hsim.Batch([big] * 64, seed=1, precision=hsim.FP32)
    assert b.layout == "replica"
    ws, sp, hi = hsim.hsim_batch_sizes(b.handle, 1, 10000)
    assert sp == 3 * 64 ** 3 * 64 * 4 and hi == 64 * 10000 * 5 * 8
    for order in (0, -1, 2048):
        b.set_order(order)
    _expect(-1, lambda: b.set_order(1))
    _expect(-1, lambda: b.set_order(-2))
    b = hsim.Batch([big], seed=1, precision=hsim.FP32)
    assert b.layout == "site"
    _expect(-6, lambda: b.set_order(0))
    _expect(-6, lambda: hsim.Batch([big] * 4, seed=0, precision=hsim.FP64_EXACT,
                                   layout=hsim.LAYOUT_REPLICA))
    _expect(-6, lambda: hsim.Batch([big, sc], seed=0, layout=hsim.LAYOUT_REPLICA))
    _expect(-1, lambda: hsim.hsim_batch_sizes(b.handle, 0, 10))
    _expect(-4, lambda: hsim.hsim_batch_run(b.handle, 0, np.ones((1, 1)), np.zeros((1, 1))))
    _expect(-4, lambda: hsim.hsim_batch_init_spins(b.handle, hsim.INIT_COLD_Z))
    _expect(-1, lambda: hsim.hsim_batch_create([], 0))


def test_site_types_and_policies_validation():
    """Site types are 0..7; every policy id and parameter is checked, and a
    batch refuses policies that leave one of its site types without a move.
    Reading the adaptive width needs a bound batch."""
    lat = synth.sc_periodic(6)
    p = hsim.Plan(lat)
    _expect(-3, lambda: p.set_types(np.full(lat.n, 8)))
    _expect(-3, lambda: p.set_types(np.full(lat.n, -1)))
    p.set_types(np.arange(lat.n) % 3)
    b = hsim.Batch([p] * 2, seed=0, precision=hsim.FP64_EXACT, layout=hsim.LAYOUT_SITE)
    R, F, S, G, H, A = (hsim.POLICY_RANDOM, hsim.POLICY_FLIP, hsim.POLICY_SMALL_STEP,
                        hsim.POLICY_GAUSSIAN, hsim.POLICY_HN, hsim.POLICY_ADAPTIVE)
    _expect(-3, lambda: b.set_policies([(R, 0.0), (F, 0.0)]))             # type 2 uncovered
    _expect(-1, lambda: b.set_policies([(R, 0.0), (F, 0.0), (9, 0.0)]))
    _expect(-3, lambda: b.set_policies([(R, 0.0), (F, 0.0), (S, 0.0)]))
    _expect(-3, lambda: b.set_policies([(R, 0.0), (F, 0.0), (H, 4.0)]))
    _expect(-3, lambda: b.set_policies([(R, 0.0), (F, 0.0), (G, -1.0)]))
    _expect(-3, lambda: b.set_policies([(R, 0.0), (F, 0.0), (A, 1.0)], sigma_min=0.0))
    _expect(-1, lambda: hsim.hsim_batch_set_policies(b.handle, [(R, 0.0)] * 9))
    b.set_policies([(R, 0.0), (S, 0.5), (A, 0.7)])
    b.set_policies([])
    _expect(-4, lambda: hsim.hsim_batch_sigma(b.handle, 2))
    p.set_types(None)


def test_energy_wrapper_rejects_mismatched_inputs():
    """The autograd wrapper hands raw pointers to kernels of the spins'
    precision, so a tensor of another dtype, shape or device is an error
    raised before any kernel runs (here checked on host tensors)."""
    import torch
    from paper_1803_07030_amd.energy import heisenberg_energy
    lat = synth.gradient_lattice(L=4, seed=4)
    plan = hsim.Plan(lat)
    n, nb = lat.n, int(plan.info.n_bonds)

    def args(dtype=torch.float32, **over):
        a = dict(spins=torch.zeros(2, 3, n, dtype=dtype), J_bond=torch.zeros(nb, dtype=dtype),
                 k=torch.zeros(n, dtype=dtype), axis=torch.zeros(3, n, dtype=dtype),
                 field_dir=None)
        a.update(over)
        return a

    def call(a):
        return heisenberg_energy(a["spins"], a["J_bond"], a["k"], torch.tensor(0.5), plan,
                                 a["axis"], a["field_dir"])

    f64 = torch.float64
    cases = [
        (TypeError, "J_bond has dtype", args(J_bond=torch.zeros(nb, dtype=f64))),
        (TypeError, "k has dtype", args(k=torch.zeros(n, dtype=f64))),
        (TypeError, "axis has dtype", args(f64, axis=torch.zeros(3, n))),
        (TypeError, "field_dir has dtype", args(field_dir=torch.zeros(3, n, dtype=f64))),
        (TypeError, "float32 or float64", args(spins=torch.zeros(2, 3, n, dtype=torch.float16))),
        (ValueError, "spins must have shape", args(spins=torch.zeros(2, n, 3))),
        (ValueError, "J_bond must have shape", args(J_bond=torch.zeros(nb + 1))),
        (ValueError, "k must have shape", args(k=torch.zeros(n - 1))),
        (ValueError, "axis must have shape", args(axis=torch.zeros(n, 3))),
        (ValueError, "field_dir must have shape", args(field_dir=torch.zeros(3, n + 2))),
        (ValueError, "must be on a CUDA device", args()),
    ]
    for exc, msg, a in cases:
        with pytest.raises(exc, match=msg):
            call(a)


def test_choose_layout_argument_errors():
    """hsim_choose_layout checks its arguments before it builds or times a
    batch (HSIM_E_ARG = -1, HSIM_E_PARAM = -3 for the schedule's values)."""
    sc = hsim.Plan(synth.sc_periodic(6))
    plans = [sc] * 4
    _expect(-1, lambda: hsim.Batch.choose_layout(plans, 1, 1.0, 0.0, trial_mcs=0))
    _expect(-3, lambda: hsim.Batch.choose_layout(plans, 1, [1.0, -0.5, 1.0, 1.0], 0.0))
    _expect(-3, lambda: hsim.Batch.choose_layout(plans, 1, [1.0, np.nan, 1.0, 1.0], 0.0))
    _expect(-3, lambda: hsim.Batch.choose_layout(plans, 1, 1.0, [0.0, 0.0, np.inf, 0.0]))
    _expect(-1, lambda: hsim.Batch.choose_layout([], 1, 1.0, 0.0))
