"""CPU tests of the host planner (through the host-only C entry point) and of
the C ABI surface: symbols, argument validation, error codes."""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

import scgen
from scgen.mesh import Subdomain

P = pytest.importorskip("paper_2509_21037_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(sc_[A-Za-z_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert {"sc_plan_create", "sc_factor", "sc_assemble", "sc_apply", "sc_apply_implicit", "sc_get_F",
            "sc_query", "sc_plan_destroy", "sc_last_error", "sc_host_analyze"} <= names
    lib = P.load()
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r"\bT (sc_\w+)", out))
    assert names <= exported


def _structural_nnz(A):
    pat = np.tril(A != 0)
    n = A.shape[0]
    for j in range(n):
        rows = np.nonzero(pat[j + 1:, j])[0] + j + 1
        if len(rows):
            pat[np.ix_(rows, rows)] |= np.tril(np.ones((len(rows), len(rows)), bool))
    return int(pat.sum())


CASES = [
    ("heat2d", lambda: scgen.config_subdomains(1)[0]),
    ("heat3d", lambda: scgen.box_subdomain("heat", (5, 6, 4), 0.2, seed=1)),
    ("elast", lambda: scgen.box_subdomain("elasticity", (3, 4, 3), 0.25, seed=2)),
    ("elast_flat", lambda: scgen.box_subdomain("elasticity", (6, 2, 3), 0.25, seed=3)),
]


@pytest.mark.parametrize("name,make", CASES)
@pytest.mark.parametrize("use_coords", [True, False])
def test_factor_is_cholesky_of_permuted_matrix(name, make, use_coords):
    s = make()
    r = P.host_analyze(s, want_L=True, use_coords=use_coords)
    perm = r["perm"]
    assert np.array_equal(np.sort(perm), np.arange(s.n))
    A = s.Kreg_csr().toarray()[np.ix_(perm, perm)]
    L = r["L"]
    assert np.abs(np.triu(L, 1)).max() == 0
    assert np.linalg.norm(L @ L.T - A) / np.linalg.norm(A) < 1e-15
    assert r["nnzL"] == _structural_nnz(A)
    assert r["nnzL_stored"] >= r["nnzL"]


def test_nested_dissection_beats_natural_order():
    s = scgen.box_subdomain("heat", (12, 12, 12), 1 / 12, seed=0)
    nd = P.host_analyze(s, values=False)
    s.perm = np.arange(s.n, dtype=np.int32)
    nat = P.host_analyze(s, values=False)
    assert nd["nnzL"] < 0.6 * nat["nnzL"]


def test_dof_blocks_stay_together_for_elasticity():
    s = scgen.box_subdomain("elasticity", (4, 3, 5), 0.25, seed=4)
    perm = P.host_analyze(s, values=False)["perm"]
    assert np.array_equal(perm.reshape(-1, 3) % 3, np.tile([0, 1, 2], (s.n // 3, 1)))
    assert np.all(perm.reshape(-1, 3)[:, 0] // 3 == perm.reshape(-1, 3)[:, 2] // 3)


@pytest.mark.parametrize("staircase", [True, False])
def test_pivots_and_column_sort(staircase):
    s = scgen.box_subdomain("heat", (6, 5, 4), 0.2, seed=7)
    r = P.host_analyze(s, values=False, staircase=staircase)
    perm, piv, pi = r["perm"], r["piv"], r["pi"]
    iperm = np.argsort(perm)
    assert np.array_equal(np.sort(pi), np.arange(s.m))
    assert np.array_equal(piv, iperm[s.dof[pi]])
    if staircase:
        assert np.all(np.diff(piv) >= 0)
        # stable: equal pivots keep the original column order
        eq = np.diff(piv) == 0
        assert np.all(np.diff(pi)[eq] > 0)
    else:
        assert np.array_equal(pi, np.arange(s.m))


def _flop_counts(L, piv, m):
    n = L.shape[0]
    c = (L != 0).sum(axis=0)
    a = np.zeros(n)
    np.add.at(a, piv, 1)
    a = np.cumsum(a)
    return float((a * (2 * c - 1)).sum()), float((a * (a + 1)).sum()), float(m * (2 * c - 1).sum()), \
        float(n * m * (m + 1))


def test_useful_flop_model_matches_definition():
    s = scgen.box_subdomain("heat", (5, 5, 5), 0.2, seed=9)
    r = P.host_analyze(s, want_L=True)
    perm = r["perm"]
    A = s.Kreg_csr().toarray()[np.ix_(perm, perm)]
    pat = np.tril(A != 0)
    for j in range(s.n):                       # structural pattern, not numerical
        rows = np.nonzero(pat[j + 1:, j])[0] + j + 1
        if len(rows):
            pat[np.ix_(rows, rows)] |= np.tril(np.ones((len(rows), len(rows)), bool))
    t, sy, td, sd = _flop_counts(pat.astype(float), r["piv"], s.m)
    assert abs(r["trsm_useful"] - t) < 1e-9 * t
    assert abs(r["syrk_useful"] - sy) < 1e-9 * sy
    assert abs(r["trsm_dense"] - td) < 1e-9 * td
    assert abs(r["syrk_dense"] - sd) < 1e-9 * sd


VISIT_CASES = [
    ("heat3d", lambda: scgen.box_subdomain("heat", (8, 8, 7), 0.2, seed=11)),
    ("elast", lambda: scgen.box_subdomain("elasticity", (5, 4, 4), 0.25, seed=12)),
    ("heat12", lambda: scgen.config_subdomains(2, count=1)[0]),
]


@pytest.mark.parametrize("split", ["uniform", "etree"])
@pytest.mark.parametrize("name,make", VISIT_CASES)
def test_trsm_visits_exactly_the_blocks_with_nonzero_rows_of_x(name, make, split):
    # X = L^{-1} P B^T solved densely: a tile must visit every block holding a
    # nonzero row of its columns (else the sweep would drop work), and with
    # random values nothing else (the reach has no cancellation)
    import scipy.linalg as sl
    s = make()
    r = P.host_analyze(s, want_L=True, block_split=split)
    row0, ptr, visit, masks = P.host_tile_visits(s, with_masks=True, block_split=split)
    L, piv, n, m = r["L"], r["piv"], s.n, s.m
    E = np.zeros((n, m))
    E[piv, np.arange(m)] = 1.0
    X = sl.solve_triangular(L, E, lower=True)
    assert row0[0] == 0 and row0[-1] == n and np.all(np.diff(row0) > 0)
    blk = np.searchsorted(row0, np.arange(n), side="right") - 1
    nt = (m + 63) // 64
    assert len(ptr) == nt + 1 and ptr[-1] == len(visit)
    stair = 0
    for t in range(nt):
        got = visit[ptr[t]:ptr[t + 1]]
        assert np.all(np.diff(got) > 0)
        rows = np.nonzero(np.abs(X[:, 64 * t:64 * t + 64]).max(axis=1) > 0)[0]
        assert np.array_equal(got, np.unique(blk[rows])), t
        # the 16-row steps marked for the tile are exactly those with a nonzero row
        steps = np.nonzero([(int(masks[t, q >> 6]) >> (q & 63)) & 1 for q in range((n + 15) // 16)])[0]
        assert np.array_equal(steps, np.unique(rows // 16)), t
        stair += len(row0) - 1 - blk[piv[64 * t]]
    assert r["trsm_visits"] == len(visit)
    assert r["stair_visits"] == stair
    # structural flop counts: r(i) = columns of X nonzero in row i, c_i from
    # the symbolic pattern of the permuted matrix
    perm = r["perm"]
    pat = np.tril(s.Kreg_csr().toarray()[np.ix_(perm, perm)] != 0)
    for j in range(n):
        below = np.nonzero(pat[j + 1:, j])[0] + j + 1
        if len(below):
            pat[np.ix_(below, below)] |= np.tril(np.ones((len(below), len(below)), bool))
    c = pat.sum(axis=0).astype(float)
    a = (X != 0).sum(axis=1).astype(float)
    t_reach, s_reach = float((a * (2 * c - 1)).sum()), float((a * (a + 1)).sum())
    assert abs(r["trsm_reach"] - t_reach) <= 1e-12 * t_reach
    assert abs(r["syrk_reach"] - s_reach) <= 1e-12 * s_reach
    assert r["trsm_reach"] <= r["trsm_useful"] and r["syrk_reach"] <= r["syrk_useful"]
    if name == "heat12":
        assert r["trsm_visits"] < 0.6 * r["stair_visits"]
    # without the reach every block from the first pivot's on; without the
    # staircase every block
    _, ptr2, visit2 = P.host_tile_visits(s, reach=False, block_split=split)
    _, ptr3, visit3 = P.host_tile_visits(s, staircase=False, block_split=split)
    for t in range(nt):
        assert np.array_equal(visit2[ptr2[t]:ptr2[t + 1]], np.arange(blk[piv[64 * t]], len(row0) - 1))
        assert np.array_equal(visit3[ptr3[t]:ptr3[t + 1]], np.arange(len(row0) - 1))


def _block_dag_depth(L, row0):
    """Levels of the block dependency DAG of the forward solve: block t
    depends on block b when L[rows of t, columns of b] has a nonzero."""
    nb = len(row0) - 1
    blk = np.searchsorted(row0, np.arange(L.shape[0]), side="right") - 1
    lev = np.zeros(nb, dtype=int)
    for b in range(nb):
        c0, c1 = row0[b], row0[b + 1]
        rows = np.nonzero(np.abs(L[c1:, c0:c1]).max(axis=1) > 0)[0] + c1
        for t in np.unique(blk[rows]):
            lev[t] = max(lev[t], lev[b] + 1)
    return int(lev.max()) + 1


@pytest.mark.parametrize("name,make", VISIT_CASES)
def test_etree_block_split(name, make):
    # blocks of at most panel_width columns that never join unrelated
    # subtrees: the block DAG of the forward solve keeps the elimination
    # tree's parallelism (far fewer levels than the uniform ranges, whose
    # blocks straddle subtrees and chain everything), and the factor is the
    # same (the split does not touch the factorisation)
    s = make()
    for bs in (32, 64):
        u = P.host_analyze(s, panel_width=bs, want_L=True)
        e = P.host_analyze(s, panel_width=bs, block_split="etree", want_L=True)
        row0, _, _ = P.host_tile_visits(s, panel_width=bs, block_split="etree")
        row0u, _, _ = P.host_tile_visits(s, panel_width=bs)
        w = np.diff(row0)
        assert row0[0] == 0 and row0[-1] == s.n and np.all(w > 0) and np.all(w <= bs)
        assert e["nblocks"] == len(w) >= u["nblocks"]
        assert e["nnzL"] == u["nnzL"] and np.array_equal(e["perm"], u["perm"])
        assert np.array_equal(e["L"], u["L"])
        d_e, d_u = _block_dag_depth(e["L"], row0), _block_dag_depth(e["L"], row0u)
        assert d_e <= d_u
        if name == "heat12":
            assert 3 * d_e < d_u and 4 * d_e <= len(w)
    with pytest.raises(P.ScasmError):
        P.host_analyze(s, block_split=2)


def test_tile_visits_capacity_error():
    s = scgen.box_subdomain("heat", (6, 5, 4), 0.2, seed=7)
    lib = P.load()
    import ctypes
    from paper_2509_21037_amd.scasm import SubdomainDesc, _fill_desc, _options
    keep = []
    d = SubdomainDesc()
    _fill_desc(d, s, keep)
    opt = _options()
    counts = np.zeros(4, dtype=np.int64)
    assert lib.sc_host_tile_visits(ctypes.byref(d), ctypes.byref(opt), counts.ctypes.data, None, None, None, 0,
                                   None) == 0
    assert counts[2] > 0 and counts[3] == (s.n + 1023) // 1024
    small = np.zeros(int(counts[2]) - 1, dtype=np.int32)
    st = lib.sc_host_tile_visits(ctypes.byref(d), ctypes.byref(opt), counts.ctypes.data, None, None,
                                 small.ctypes.data, int(counts[2]) - 1, None)
    assert st == P.SC_ERR_INVALID_ARG and b"capacity" in lib.sc_last_error()
    assert lib.sc_host_tile_visits(ctypes.byref(d), ctypes.byref(opt), None, None, None, None, 0, None) == \
        P.SC_ERR_INVALID_ARG


def test_triangular_rhs_gives_threefold_saving():
    # Sec. 4.3: pivot of column j at row j*n/m with a dense factor -> 1/3 of the work
    golden = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_values.txt")):
        if line.strip() and not line.startswith("#"):
            k, v, _ = line.split()
            golden[k] = float(v)
    n = m = 1000
    rng = np.random.default_rng(0)
    M = rng.standard_normal((n, n))
    Kd = M @ M.T + n * np.eye(n)
    rowptr = np.arange(0, n * n + 1, n, dtype=np.int64)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    sd = Subdomain(kind="dense", dim=0, elems=(), h=1.0, dofs_per_node=1, n=n, k_rowptr=rowptr, k_col=col,
                   k_val=Kd.ravel(), rowptr=rowptr, col=col, val=Kd.ravel(), coords=None, R=np.zeros((n, 0)),
                   fix_dofs=np.zeros(0, int), Q=np.zeros((0, 0)), rho=0.0,
                   dof=(np.arange(m) * n // m).astype(np.int32), sign=np.ones(m, np.int8))
    sd.perm = np.arange(n, dtype=np.int32)
    r = P.host_analyze(sd, values=False)
    ratio_trsm = r["trsm_dense"] / r["trsm_useful"]
    ratio_syrk = r["syrk_dense"] / r["syrk_useful"]
    assert abs(ratio_trsm - golden["triangular_rhs_speedup"]) < 0.1
    assert abs(ratio_syrk - golden["triangular_rhs_speedup"]) < 0.1


def test_not_spd_reported_with_column():
    s = scgen.box_subdomain("heat", (3, 3, 3), 0.3, seed=1)
    bad = Subdomain(**{**s.__dict__})
    bad.val = s.k_val            # K itself is singular (floating subdomain)
    bad.rowptr, bad.col = s.k_rowptr, s.k_col
    with pytest.raises(P.ScasmError) as e:
        P.host_analyze(bad)
    assert e.value.status == P.SC_ERR_NOT_SPD
    assert 0 <= e.value.failed_col < s.n


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: setattr(s, "dof", np.concatenate([s.dof[:-1], [s.n]]).astype(np.int32)), "dof"),
    (lambda s: setattr(s, "dof", np.concatenate([s.dof[:-1], [-1]]).astype(np.int32)), "dof"),
    (lambda s: setattr(s, "sign", np.concatenate([s.sign[:-1], [2]]).astype(np.int8)), "sign"),
    (lambda s: setattr(s, "sign", np.concatenate([s.sign[:-1], [0]]).astype(np.int8)), "sign"),
    (lambda s: setattr(s, "perm", np.zeros(s.n, np.int32)), "perm"),
    (lambda s: setattr(s, "col", np.where(np.arange(len(s.col)) == 3, s.n, s.col).astype(np.int32)), "column"),
    # rejected before the pattern is read (the step entries of the SYRK hold
    # a row below 2^27)
    (lambda s: setattr(s, "n", 1 << 27), "2^27"),
])
def test_invalid_arguments(mutate, msg):
    s = scgen.box_subdomain("heat", (3, 3), 0.3, seed=1)
    bad = Subdomain(**{**s.__dict__})
    mutate(bad)
    with pytest.raises(P.ScasmError) as e:
        P.host_analyze(bad, values=False)
    assert e.value.status == P.SC_ERR_INVALID_ARG
    assert msg in e.value.message


def test_invalid_options_and_sizes():
    s = scgen.box_subdomain("heat", (3, 3), 0.3, seed=1)
    for kw in ({"panel_width": 8}, {"panel_width": 128}, {"precision": 7}, {"relax_width": -1}):
        with pytest.raises(P.ScasmError) as e:
            P.host_analyze(s, values=False, **kw)
        assert e.value.status == P.SC_ERR_INVALID_ARG
    bad = Subdomain(**{**s.__dict__})
    bad.n = 0
    with pytest.raises(P.ScasmError):
        P.host_analyze(bad, values=False)


def test_plan_create_validates_before_touching_the_device():
    lib = P.load()
    from paper_2509_21037_amd.scasm import Options
    h = ctypes.c_void_p(0)
    assert lib.sc_plan_create(None, 1, ctypes.byref(Options()), None, ctypes.byref(h)) == P.SC_ERR_INVALID_ARG
    assert lib.sc_plan_create(None, -1, None, None, ctypes.byref(h)) == P.SC_ERR_INVALID_ARG
    assert lib.sc_plan_create(None, 0, None, None, None) == P.SC_ERR_INVALID_ARG
    assert lib.sc_assemble(None, None) == P.SC_ERR_INVALID_ARG
    assert lib.sc_plan_destroy(None) == P.SC_OK
    assert b"NULL" in lib.sc_last_error() or lib.sc_last_error() == b""


def test_arena_cap_below_one_subdomain_is_oom_before_the_device():
    # temporary-memory waves: a cap below the X slabs of one subdomain is
    # refused with SC_ERR_OOM at plan creation, before any device call (this
    # machine has no device); overlapped assembly cannot run in waves
    subs = scgen.config_subdomains(3, count=2)
    with pytest.raises(P.ScasmError) as e:
        P.Plan(subs, arena_cap_bytes=4096)
    assert e.value.status == P.SC_ERR_OOM and "arena_cap_bytes" in str(e.value)
    with pytest.raises(P.ScasmError) as e:
        P.Plan(subs, arena_cap_bytes=1 << 40, assembly="overlap")
    assert e.value.status == P.SC_ERR_UNSUPPORTED
    with pytest.raises(P.ScasmError) as e:
        P.Plan(subs, arena_cap_bytes=-1)
    assert e.value.status == P.SC_ERR_INVALID_ARG


@pytest.mark.parametrize("bad", [{"panel_width": 8}, {"block_split": 2}, {"syrk_kind": 3},
                                 {"n_lo": 10, "n_hi": 5}])
def test_tune_classes_are_validated_before_the_device(bad):
    cls = {"n_lo": 0, "n_hi": 1 << 30, "panel_width": 32, "block_split": 1, "syrk_kind": 1}
    cls.update(bad)
    with pytest.raises(P.ScasmError) as e:
        P.Plan(scgen.config_subdomains(1), tune_classes=[cls])
    assert e.value.status == P.SC_ERR_INVALID_ARG and "tune class" in str(e.value)


def test_selection_prediction_follows_its_model():
    # per-subdomain explicit / implicit choice (select_iters): t_asm from the
    # structural flops, t_expl from the stored F bytes, t_impl from 16 nnz(L)
    # bytes, n* = t_asm / (t_impl - t_expl)
    for s in (scgen.config_subdomains(2, count=1)[0], scgen.config_subdomains(3, count=1)[0]):
        for prec, sF in (("fp64", 8), ("mixed", 4)):
            r = P.host_analyze(s, values=False, precision=prec, select_model=(10.0, 2000.0, 500.0))
            nst = (s.m + 127) // 128
            assert np.isclose(r["t_asm_ms"], (r["trsm_reach"] + r["syrk_reach"]) / 10e12 * 1e3)
            assert np.isclose(r["t_expl_ms"], nst * (nst + 1) / 2 * 128 * 128 * sF / 2000e9 * 1e3)
            assert np.isclose(r["t_impl_ms"], 16 * r["nnzL"] / 500e9 * 1e3)
            assert np.isclose(r["n_star"], r["t_asm_ms"] / (r["t_impl_ms"] - r["t_expl_ms"]))
        fast = P.host_analyze(s, values=False, select_model=(10.0, 2000.0, 1e9))
        assert fast["n_star"] == float("inf")          # the implicit apply never loses
        d = P.host_analyze(s, values=False)            # default rates
        assert d["t_asm_ms"] > 0 and d["t_impl_ms"] > 0
    with pytest.raises(P.ScasmError):
        P.host_analyze(s, values=False, select_iters=-1)


def _lower_only(s):
    """The same subdomain with only the CSR entries on and below the diagonal."""
    import copy
    keep = np.repeat(np.arange(s.n), np.diff(s.rowptr)) >= s.col
    t = copy.copy(s)
    t.col = s.col[keep]
    t.val = s.val[keep]
    t.rowptr = np.concatenate([[0], np.cumsum(np.add.reduceat(keep.astype(np.int64), s.rowptr[:-1])
                                               * (np.diff(s.rowptr) > 0))]).astype(np.int64)
    assert t.rowptr[-1] == keep.sum()
    return t


@pytest.mark.parametrize("make", [lambda: scgen.config_subdomains(1)[0],
                                  lambda: scgen.box_subdomain("elasticity", (4, 3, 5), 0.25, seed=8),
                                  lambda: scgen.paper_subdomains(3, 9, count=1)[0]])
def test_lower_only_csr_gives_the_same_plan_and_factor(make):
    s = make()
    lo = _lower_only(s)
    assert len(lo.col) < len(s.col)
    full = P.host_analyze(s, want_L=True)
    low = P.host_analyze(lo, want_L=True, lower_only_csr=True)
    assert np.array_equal(full["perm"], low["perm"]) and np.array_equal(full["piv"], low["piv"])
    assert full["nnzL"] == low["nnzL"] and full["nblocks"] == low["nblocks"]
    # the same pattern; the values agree to rounding (a full CSR assembled
    # in floating point is symmetric only to rounding, and the full-pattern
    # run takes each pair's entry from the row that comes later in the order)
    assert np.array_equal(full["L"] != 0, low["L"] != 0)
    assert np.abs(full["L"] - low["L"]).max() <= 1e-13 * np.abs(full["L"]).max()
    # an entry above the diagonal is refused in that mode
    with pytest.raises(P.ScasmError) as e:
        P.host_analyze(s, values=False, lower_only_csr=True)
    assert e.value.status == P.SC_ERR_INVALID_ARG and "above the diagonal" in str(e.value)


def test_options_struct_matches_the_c_header(tmp_path):
    # ctypes layout of sc_options_t, sc_subdomain_desc_t, sc_tune_class_t and
    # sc_host_info_t against the C compiler's (sizes and field offsets)
    import ctypes
    from paper_2509_21037_amd.scasm import HostInfo, Options, SubdomainDesc, TuneClass
    fields = {"sc_options_t": Options, "sc_subdomain_desc_t": SubdomainDesc, "sc_tune_class_t": TuneClass,
              "sc_host_info_t": HostInfo}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "scasm_host.h"', "int main(void) {"]
    for cname, py in fields.items():
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "abi.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "abi"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.run([str(exe)], stdout=subprocess.PIPE, text=True,
                                                       check=True).stdout.splitlines())
    for cname, py in fields.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_merged_block_pairs_of_the_trsm():
    """Pairs of factor blocks whose TRSM updates below merge (the first
    block's rows below are the second block's rows followed by its rows
    below): present on the 20^3 elasticity subdomain with both splits, none
    when disabled or on the 16 x 16 heat subdomain (5 blocks, no consecutive
    two of them nested that way); the saved updates are
    at most half the pruned rows of the blocks the tiles visit."""
    s = scgen.config_subdomains(5, count=1)[0]
    for split in ("uniform", "etree"):
        h = P.host_analyze(s, values=False, block_split=split)
        assert h["merge_pairs"] > 10 and h["merged_rows"] > 0
        off = P.host_analyze(s, values=False, block_split=split, pair_merge=False)
        assert off["merge_pairs"] == 0 and off["merged_rows"] == 0
        # a merged update replaces two: at most half of all updates are saved
        assert off["pruned_updates"] == h["pruned_updates"] > 0
        assert 2 * h["merged_rows"] <= h["pruned_updates"]
    tiny = scgen.config_subdomains(1)[0]
    assert P.host_analyze(tiny, values=False)["merge_pairs"] == 0


def test_zero_multipliers_and_tiny_subdomain():
    s = scgen.box_subdomain("heat", (1, 1), 1.0, seed=1)
    r = P.host_analyze(s, want_L=True)
    assert r["n"] == 4
    e = Subdomain(**{**s.__dict__})
    e.dof = np.zeros(0, np.int32)
    e.sign = np.zeros(0, np.int8)
    r = P.host_analyze(e)
    assert r["m"] == 0 and r["trsm_useful"] == 0 and r["syrk_useful"] == 0


def test_dual_vector_checks_reject_bad_tensors_before_any_call():
    import torch
    n = 50
    good = torch.zeros(n, dtype=torch.float64)
    cases = [
        (np.zeros(n), "must be a torch.Tensor"),
        (torch.zeros(n, dtype=torch.float32), "must be float64"),
        (torch.zeros(2 * n, dtype=torch.float64)[::2], "must be contiguous"),
        (torch.zeros(n - 1, dtype=torch.float64), "elements, the plan's dual vectors have"),
        (good, "must be a device tensor"),
    ]
    for t, msg in cases:
        with pytest.raises(P.ScasmError) as e:
            P.check_dual_tensor(t, n, 0, "p")
        assert e.value.status == P.SC_ERR_INVALID_ARG
        assert msg in e.value.message, (msg, e.value.message)
