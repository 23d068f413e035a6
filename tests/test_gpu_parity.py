"""Parity of the HIP assembly (through the C ABI) with the CPU oracle.

F_gpu from sc_assemble (FP64 path) is compared element by element with the
long-double oracle F = B K_reg^{-1} B^T on the same seeded inputs; the bar is
a relative Frobenius error <= 1e-12 per subdomain.  At the full workload sizes
the comparison uses seeded column subsets S (F[S, S]) the oracle computes on
its own."""
import os

import numpy as np
import pytest

import oracle
import scgen
from scgen.rng import signs_from_seed, stream_seed

P = pytest.importorskip("paper_2509_21037_amd")
pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


def _torch_init():
    import torch
    assert torch.cuda.is_available()
    torch.cuda.init()
    return torch


def _assemble(subs, **kw):
    _torch_init()
    plan = P.Plan(subs, **kw)
    plan.factor()
    plan.assemble()
    return plan


def _check_against_oracle(plan, subs, max_full=3000, nsel=192, seed=0):
    errs = []
    for i, s in enumerate(subs):
        F = plan.get_F(i)
        assert F.shape == (s.m, s.m)
        if s.m == 0:
            continue
        assert np.array_equal(F, F.T)
        if s.n <= max_full:
            ref = oracle.schur(s)
            e = oracle.relF(F, ref)
        else:
            sel = np.sort(np.random.default_rng(seed + i).choice(s.m, size=min(nsel, s.m), replace=False))
            ref = oracle.schur(s, sel=sel)
            e = oracle.relF(F[np.ix_(sel, sel)], ref)
        errs.append(e)
        assert e <= TOL_FP64, (i, s.elems, e)
    return errs


def test_heat2d_matches_golden_and_oracle():
    s = scgen.config_subdomains(1)[0]
    plan = _assemble([s])
    F = plan.get_F(0)
    import os
    golden = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "heat2d_q1_16x16_F.txt"),
                        comments="#").reshape(s.m, s.m, order="F")
    assert oracle.relF(F, golden) <= TOL_FP64
    _check_against_oracle(plan, [s])


def test_heat3d_batch_matches_oracle():
    subs = scgen.config_subdomains(2, count=3)
    plan = _assemble(subs)
    _check_against_oracle(plan, subs)


def test_elasticity_uneven_batch_matches_oracle():
    subs = scgen.config_subdomains(3, count=6)
    plan = _assemble(subs)
    _check_against_oracle(plan, subs, max_full=3000)


@pytest.mark.parametrize("panel_width", [16, 32, 48, 64])
def test_panel_widths(panel_width):
    subs = [scgen.box_subdomain("elasticity", (4, 5, 3), 0.25, seed=5),
            scgen.box_subdomain("heat", (7, 6, 5), 0.2, seed=6)]
    plan = _assemble(subs, panel_width=panel_width, relax_width=96)
    _check_against_oracle(plan, subs)


@pytest.mark.parametrize("panel_width", [16, 32, 48])
def test_panel_widths_mixed(panel_width):
    subs = [scgen.box_subdomain("elasticity", (4, 5, 3), 0.25, seed=5),
            scgen.box_subdomain("heat", (7, 6, 5), 0.2, seed=6)]
    plan = _assemble(subs, precision="mixed", panel_width=panel_width, relax_width=96)
    for i, s in enumerate(subs):
        assert oracle.relF(plan.get_F(i), oracle.schur(s)) <= 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_get_F_on_device_equals_host_copy(precision):
    """sc_get_F(on_device = 1) writes the same FP64 values as the host copy,
    with a leading dimension larger than m and the padding left untouched."""
    torch = _torch_init()
    subs = scgen.config_subdomains(3, count=2) + [scgen.config_subdomains(1)[0]]
    plan = _assemble(subs, precision=precision)
    for i, s in enumerate(subs):
        ld = s.m + 3
        out = torch.full((ld * s.m,), 7.0, dtype=torch.float64, device="cuda")
        Fd = plan.get_F_device(i, out=out, ld=ld)
        assert np.array_equal(Fd.cpu().numpy(), plan.get_F(i))
        pad = out.view(s.m, ld)[:, s.m:]
        assert bool((pad == 7.0).all())


def test_full_uneven_elasticity_largest_subdomain_whole_F():
    """The largest subdomain of the 512-box elasticity batch (16 x 15 x 16
    elements, n = 13872, m = 4422) in the whole-batch assembly, against the
    whole F of the long-double oracle."""
    subs = scgen.config_subdomains(3)
    big = int(np.argmax([s.n for s in subs]))
    s = subs[big]
    assert (s.n, s.m) == (13872, 4422)
    plan = _assemble(subs)
    F = plan.get_F(big)
    plan.destroy()
    assert np.array_equal(F, F.T)
    assert oracle.relF(F, oracle.schur(s)) <= TOL_FP64


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_large_elasticity_512_columns_direct(precision):
    """The 64 x 20^3 elasticity batch in one assembly; 512 seeded columns of
    two subdomains, each computed directly by the long-double oracle with that
    subdomain's own signs (no sign-flip relation)."""
    subs = scgen.config_subdomains(5)
    plan = _assemble(subs, precision=precision, use_graph=True)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    for k in (0, 45):
        s = subs[k]
        sel = np.sort(np.random.default_rng(500 + k).choice(s.m, size=512, replace=False))
        F = plan.get_F(k)[np.ix_(sel, sel)]
        assert oracle.relF(F, oracle.schur(s, sel=sel)) <= tol, k
    plan.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_etree_block_split_matches_oracle(precision):
    """Factor blocks that follow the elimination tree (non-uniform widths,
    Sec. 4.1 footnote) in the TRSM and SYRK: against the oracle, and equal to
    the uniform split within rounding."""
    subs = scgen.config_subdomains(2, count=2) + scgen.config_subdomains(3, count=4) + \
        scgen.paper_subdomains(3, 14, count=1)
    plan = _assemble(subs, precision=precision, block_split="etree")
    uni = _assemble(subs, precision=precision)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    for i, s in enumerate(subs):
        F = plan.get_F(i)
        assert np.array_equal(F, F.T)
        assert oracle.relF(F, uni.get_F(i)) <= (1e-13 if precision == "fp64" else 1e-6)
        if s.n <= 3000:
            assert oracle.relF(F, oracle.schur(s)) <= tol, i
        else:
            sel = np.sort(np.random.default_rng(i).choice(s.m, size=min(128, s.m), replace=False))
            assert oracle.relF(F[np.ix_(sel, sel)], oracle.schur(s, sel=sel)) <= tol, i
    plan.destroy()
    uni.destroy()


def test_lower_only_csr_and_plan_wide_syrk_kind():
    """A plan fed the lower triangle of K_reg (lower_only_csr) assembles the
    F of the full-pattern plan to rounding; the SYRK as 64 x 64 blocks or as
    128 x 128 tiles for every subdomain gives the same F to rounding."""
    from test_planner_abi import _lower_only
    subs = scgen.config_subdomains(3, count=3) + scgen.config_subdomains(1)
    full = _assemble(subs)
    low = _assemble([_lower_only(s) for s in subs], lower_only_csr=True)
    for i, s in enumerate(subs):
        assert oracle.relF(low.get_F(i), full.get_F(i)) <= 1e-13
    for kind in (1, 2):
        k = _assemble(subs, syrk_kind=kind)
        for i in range(len(subs)):
            assert oracle.relF(k.get_F(i), full.get_F(i)) <= 1e-13, (kind, i)
        k.destroy()
    full.destroy()
    low.destroy()


def test_staircase_off_matches_on():
    subs = [scgen.config_subdomains(1)[0], scgen.box_subdomain("elasticity", (4, 3, 5), 0.25, seed=8)]
    on = _assemble(subs)
    off = _assemble(subs, staircase=False)
    for i in range(len(subs)):
        a, b = on.get_F(i), off.get_F(i)
        assert oracle.relF(a, b) <= 1e-14
    _check_against_oracle(off, subs)


def test_sign_flip_is_exact():
    s = scgen.box_subdomain("heat", (6, 6, 6), 1 / 6, seed=11)
    flip = scgen.rng.signs_from_seed(5, s.m).astype(np.int8)
    plan = _assemble([s, s.with_signs(s.sign * flip)])
    F0, F1 = plan.get_F(0), plan.get_F(1)
    S = flip.astype(float)
    assert np.array_equal(F1, S[:, None] * F0 * S[None, :])


def test_column_permutation():
    s = scgen.box_subdomain("elasticity", (3, 4, 4), 0.25, seed=12)
    perm = np.random.default_rng(1).permutation(s.m)
    plan = _assemble([s, s.with_columns(s.dof[perm], s.sign[perm])])
    F0, F1 = plan.get_F(0), plan.get_F(1)
    assert oracle.relF(F1, F0[np.ix_(perm, perm)]) <= 1e-14


def test_run_to_run_deterministic():
    subs = scgen.config_subdomains(3, count=2)
    plan = _assemble(subs)
    a = [plan.get_F(i) for i in range(2)]
    plan.assemble()
    b = [plan.get_F(i) for i in range(2)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("assembly", ["overlap", "separate"])
def test_edge_cases_in_one_batch(assembly):
    base = scgen.box_subdomain("heat", (4, 4, 3), 0.25, seed=13)
    tiny = scgen.box_subdomain("heat", (1, 1), 1.0, seed=14)            # n = 4, m = 4
    empty = base.with_columns(np.zeros(0, np.int32), np.zeros(0, np.int8))
    one = base.with_columns(base.dof[:1], base.sign[:1])
    ragged = base.with_columns(base.dof[:17], base.sign[:17])
    same_pivot = base.with_columns(np.full(70, base.dof[5], np.int32),
                                   scgen.rng.signs_from_seed(3, 70))   # 70 columns, one DOF
    interior = base.with_columns(np.arange(0, base.n, 7, dtype=np.int32),
                                 scgen.rng.signs_from_seed(4, len(range(0, base.n, 7))))
    subs = [base, tiny, empty, one, ragged, same_pivot, interior]
    plan = _assemble(subs, assembly=assembly)
    _check_against_oracle(plan, subs)


def test_state_errors():
    _torch_init()
    s = scgen.config_subdomains(1)[0]
    plan = P.Plan([s])
    with pytest.raises(P.ScasmError) as e:
        plan.assemble()
    assert e.value.status == P.SC_ERR_STATE
    with pytest.raises(P.ScasmError) as e:
        plan.get_F(0)
    assert e.value.status == P.SC_ERR_STATE
    with pytest.raises(P.ScasmError) as e:
        plan.get_F(5)
    assert e.value.status == P.SC_ERR_INVALID_ARG


def test_not_spd_from_factor():
    _torch_init()
    s = scgen.box_subdomain("heat", (3, 3, 3), 0.3, seed=1)
    plan = P.Plan([s, s])
    with pytest.raises(P.ScasmError) as e:
        plan.factor([s.val, np.where(np.arange(len(s.val)) == 0, -1.0, s.val)])
    assert e.value.status == P.SC_ERR_NOT_SPD and e.value.failed_sub == 1


def test_full_heat_workload_sampled():
    """All 1024 subdomains of the 12^3 heat workload in one assembly (the
    launch the benchmark times); three subdomains checked in full."""
    subs = scgen.config_subdomains(2)
    plan = _assemble(subs)
    for i in (0, 511, 1023):
        F = plan.get_F(i)
        assert oracle.relF(F, oracle.schur(subs[i])) <= TOL_FP64


def test_full_elasticity_workload_sampled():
    """All 512 uneven elasticity subdomains in one assembly; seeded column
    samples of four subdomains (the largest included) against the oracle."""
    subs = scgen.config_subdomains(3)
    plan = _assemble(subs)
    sizes = np.array([s.n for s in subs])
    picks = [0, int(np.argmax(sizes)), int(np.argmin(sizes)), 300]
    for i in picks:
        s = subs[i]
        sel = np.sort(np.random.default_rng(i).choice(s.m, size=min(128, s.m), replace=False))
        F = plan.get_F(i)
        assert oracle.relF(F[np.ix_(sel, sel)], oracle.schur(s, sel=sel)) <= TOL_FP64


def _large_workload_sample():
    """The 64 x 20^3 elasticity batch (one mesh, per-subdomain signs) and the
    stored oracle sample F_0[S, S] of its subdomain 0."""
    path = os.path.join(os.path.dirname(__file__), "golden", "elast3d_hex8_20cube_F_sample.txt")
    with open(path) as f:
        f.readline()
        sel = np.array([int(v) for v in f.readline().split()], dtype=np.int64)
    F0 = np.loadtxt(path, comments="#", skiprows=2).reshape(len(sel), len(sel), order="F")
    s0 = scgen.config_subdomains(5, count=1)[0]
    base = scgen.BASE_SEED + 5
    subs = [s0] + [s0.with_signs(signs_from_seed(stream_seed(base, i), s0.m)) for i in range(1, 64)]
    return subs, sel, F0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_large_elasticity_workload_sampled(precision):
    """All 64 subdomains of the 20^3 elasticity workload (n = 27783, m = 7938)
    in one assembly, as the benchmark launches it (captured graph); sampled
    columns of four subdomains against the stored oracle sample.  The
    subdomains share K and the multiplier DOFs, so F_k[S, S] = D F_0[S, S] D
    with D = diag(sign_k sign_0)[S] exactly."""
    subs, sel, F0 = _large_workload_sample()
    plan = _assemble(subs, precision=precision, use_graph=True)
    plan.assemble()
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    for k in (0, 21, 42, 63):
        d = (subs[k].sign.astype(np.float64) * subs[0].sign)[sel]
        F = plan.get_F(k)[np.ix_(sel, sel)]
        assert oracle.relF(F, d[:, None] * F0 * d[None, :]) <= tol, k
    if precision == "fp64":
        # the implicit apply of the whole batch (its bottom levels hold
        # thousands of blocks) against the explicit apply of the checked F
        torch = _torch_init()
        p, _ = _dual_vectors(plan, subs, seed=23)
        qi, qe = torch.zeros_like(p), torch.zeros_like(p)
        plan.apply(p, qe)
        plan.apply_implicit(p, qi)
        for k in range(len(subs)):
            o = plan.query(k)["dual_offset"]
            a, b = qi[o:o + subs[k].m], qe[o:o + subs[k].m]
            assert float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) <= 1e-12, k
    plan.destroy()


def _dual_vectors(plan, subs, seed=0):
    import torch
    st = plan.stats()
    p = torch.from_numpy(scgen.splitmix64_uniform(seed, st["dual_total"])).cuda()
    q = torch.zeros_like(p)
    return p, q


@pytest.mark.parametrize("cfg,count", [(1, 1), (2, 3), (3, 5)])
def test_explicit_apply_matches_dense_product(cfg, count):
    subs = scgen.config_subdomains(cfg, count=count)
    odd = scgen.box_subdomain("heat", (3, 4, 2), 0.25, seed=3)
    odd = odd.with_columns(odd.dof[:33], odd.sign[:33])          # odd m: unaligned column starts
    subs = subs + [odd]
    plan = _assemble(subs)
    p, q = _dual_vectors(plan, subs)
    plan.apply(p, q)
    qh = q.cpu().numpy()
    ph = p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        ref = oracle.schur(s) @ ph[o:o + s.m]
        got = qh[o:o + s.m]
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), i


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_apply_is_deterministic_and_symmetric_storage_complete(precision):
    """The two-pass apply over the stored lower tiles gives the same bits on
    every call, and equals get_F(i) @ p (get_F expands the same tiles)."""
    subs = scgen.config_subdomains(3, count=5)            # m 654 .. 4614: several 128-tiles, ragged
    plan = _assemble(subs, precision=precision)
    p, q = _dual_vectors(plan, subs, seed=11)
    plan.apply(p, q)
    q1 = q.clone()
    for _ in range(3):
        q.zero_()
        plan.apply(p, q)
        assert bool((q == q1).all())
    qh, ph = q.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        ref = plan.get_F(i) @ ph[o:o + s.m]
        assert np.linalg.norm(qh[o:o + s.m] - ref) <= 1e-13 * np.linalg.norm(ref), i


def test_apply_state_and_alias_errors():
    torch = _torch_init()
    s = scgen.config_subdomains(1)[0]
    plan = P.Plan([s])
    plan.factor()
    p = torch.zeros(s.m, dtype=torch.float64, device="cuda")
    with pytest.raises(P.ScasmError) as e:
        plan.apply(p, torch.zeros_like(p))
    assert e.value.status == P.SC_ERR_STATE
    plan.assemble()
    with pytest.raises(P.ScasmError) as e:
        plan.apply(p, p)
    assert e.value.status == P.SC_ERR_INVALID_ARG


def test_wrong_dual_tensors_are_rejected_before_any_launch():
    """FP32, short, strided and host tensors never reach the kernels of the
    explicit apply, the implicit apply or PCPG."""
    torch = _torch_init()
    s = scgen.config_subdomains(1)[0]
    plan = P.Plan([s])
    plan.factor()
    plan.assemble()
    good = torch.zeros(s.m, dtype=torch.float64, device="cuda")
    bad = [torch.zeros(s.m, dtype=torch.float32, device="cuda"),
           torch.zeros(s.m - 1, dtype=torch.float64, device="cuda"),
           torch.zeros(2 * s.m, dtype=torch.float64, device="cuda")[::2],
           torch.zeros(s.m, dtype=torch.float64)]
    for b in bad:
        for f in (plan.apply, plan.apply_implicit):
            for args in ((b, good), (good, b)):
                with pytest.raises(P.ScasmError) as e:
                    f(*args)
                assert e.value.status == P.SC_ERR_INVALID_ARG
        with pytest.raises(P.ScasmError) as e:
            plan.pcpg(b, good, 3)
        assert e.value.status == P.SC_ERR_INVALID_ARG
    torch.cuda.synchronize()
    plan.destroy()


# ---------------------------------------------------------------- mixed precision

TOL_MIXED = 1e-5


@pytest.mark.parametrize("cfg,count", [(1, 1), (2, 3), (3, 6)])
def test_mixed_precision_matches_oracle(cfg, count):
    subs = scgen.config_subdomains(cfg, count=count)
    plan = _assemble(subs, precision="mixed")
    for i, s in enumerate(subs):
        F = plan.get_F(i)
        assert np.array_equal(F, F.T)
        if s.n <= 3000:
            e = oracle.relF(F, oracle.schur(s))
        else:
            sel = np.sort(np.random.default_rng(i).choice(s.m, size=192, replace=False))
            e = oracle.relF(F[np.ix_(sel, sel)], oracle.schur(s, sel=sel))
        assert e <= TOL_MIXED, (i, s.elems, e)


def test_mixed_apply_reads_fp32_accumulates_fp64():
    subs = scgen.config_subdomains(3, count=3)
    plan = _assemble(subs, precision="mixed")
    p, q = _dual_vectors(plan, subs, seed=7)
    plan.apply(p, q)
    qh, ph = q.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        F = plan.get_F(i)                      # the stored FP32 values, widened
        ref = F @ ph[o:o + s.m]
        assert np.linalg.norm(qh[o:o + s.m] - ref) <= 1e-13 * np.linalg.norm(ref)


# ---------------------------------------------------------------- PCPG

def _pcpg_case(precision, cfg=3, count=4, iters=30):
    import torch
    subs = scgen.config_subdomains(cfg, count=count)
    plan = _assemble(subs, precision=precision)
    st = plan.stats()
    d = torch.from_numpy(scgen.splitmix64_uniform(scgen.BASE_SEED + 4, st["dual_total"])).cuda()
    lam = torch.zeros_like(d)
    hist = plan.pcpg(d, lam, iters, history=True)
    return subs, plan, d.cpu().numpy(), lam.cpu().numpy(), hist


def test_pcpg_fp64_matches_oracle():
    # Compared at convergence (100 iterations, as in the mixed workload): in
    # mid-run, CG amplifies round-off-level differences of F by many orders
    # (two oracle F differing by 2e-14 give lambda 5e-8..1e-5 apart at 30
    # iterations, 2e-14 apart at 100).
    iters = 100
    subs, plan, d, lam, hist = _pcpg_case("fp64", iters=iters)
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        F = oracle.schur(s)
        ref, href = oracle.pcpg(F, oracle.gluing_G(s), d[o:o + s.m], iters)
        assert np.linalg.norm(lam[o:o + s.m] - ref) <= 1e-10 * np.linalg.norm(ref), i
        assert abs(hist[0, i] - href[0]) <= 1e-12 * href[0]
        assert hist[-1, i] < 1e-10 * hist[0, i]


def test_pcpg_mixed_close_to_fp64():
    iters = 100
    _, plan64, d, lam64, _ = _pcpg_case("fp64", iters=iters)
    _, plan32, _, lam32, _ = _pcpg_case("mixed", iters=iters)
    err = np.linalg.norm(lam32 - lam64) / np.linalg.norm(lam64)
    assert err < 1e-3, err


# ---------------------------------------------------------------- implicit apply

@pytest.mark.parametrize("split", ["uniform", "etree"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_implicit_apply_matches_oracle(precision, split):
    base = scgen.box_subdomain("heat", (4, 4, 3), 0.25, seed=13)
    per_face = scgen.box_subdomain("elasticity", (3, 2, 3), 0.25, seed=15, gluing="per_face")
    subs = scgen.config_subdomains(1) + scgen.config_subdomains(3, count=3) + [base, per_face]
    _torch_init()
    plan = P.Plan(subs, precision=precision, block_split=split)
    plan.factor()
    p, q = _dual_vectors(plan, subs, seed=11)
    plan.apply_implicit(p, q)            # needs only the factor (before sc_assemble)
    qh, ph = q.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        if s.n <= 3000:
            ref = oracle.schur(s) @ ph[o:o + s.m]
        else:
            import scipy.sparse.linalg as spla
            Bt = s.Bt_dense()
            ref = Bt.T @ spla.spsolve(s.Kreg_csr().tocsc(), Bt @ ph[o:o + s.m])
        assert np.linalg.norm(qh[o:o + s.m] - ref) <= 1e-12 * np.linalg.norm(ref), i


@pytest.mark.parametrize("split", ["uniform", "etree"])
def test_implicit_apply_on_large_subdomains_matches_explicit(split):
    """Two 20^3 elasticity subdomains (n = 27783, blocks with up to ~1300
    pruned rows at the top of the elimination tree): the implicit apply
    against the explicit apply of the assembled F, eagerly and as graph
    replays, three calls in a row."""
    torch = _torch_init()
    subs = scgen.config_subdomains(5, count=2)
    for graph in (False, True):
        plan = _assemble(subs, block_split=split, use_graph=graph)
        p, _ = _dual_vectors(plan, subs, seed=31)
        qi, qe = torch.zeros_like(p), torch.zeros_like(p)
        plan.apply(p, qe)
        for _ in range(3):
            plan.apply_implicit(p, qi)
            torch.cuda.synchronize()
            assert float(torch.linalg.norm(qi - qe) / torch.linalg.norm(qe)) <= 1e-12
        plan.destroy()


def _block_diagonal_subdomain(ncomp, bs, m, seed):
    """K_reg = block diagonal of ncomp random SPD bs x bs blocks (a forest of
    independent components), m multipliers on random DOFs, identity order."""
    from scgen.mesh import Subdomain
    rng = np.random.default_rng(seed)
    n = ncomp * bs
    K = np.zeros((n, n))
    for c in range(ncomp):
        M = rng.standard_normal((bs, bs))
        K[c * bs:(c + 1) * bs, c * bs:(c + 1) * bs] = M @ M.T + bs * np.eye(bs)
    rows, cols = np.nonzero(K)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    col = cols.astype(np.int32)
    val = K[rows, cols]
    dof = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    sd = Subdomain(kind="dense", dim=0, elems=(), h=1.0, dofs_per_node=1, n=n, k_rowptr=rowptr, k_col=col,
                   k_val=val, rowptr=rowptr, col=col, val=val, coords=None, R=np.zeros((n, 0)),
                   fix_dofs=np.zeros(0, int), Q=np.zeros((0, 0)), rho=0.0, dof=dof,
                   sign=scgen.rng.signs_from_seed(seed, m))
    sd.perm = np.arange(n, dtype=np.int32)
    return sd


def test_implicit_apply_level_launches_on_a_forest():
    """Subdomains whose factor blocks are independent (many blocks per
    elimination level) take the one-launch-per-level sweeps instead of one
    workgroup per subdomain; against the oracle."""
    _torch_init()
    subs = [_block_diagonal_subdomain(40, 16, 64, seed=31 + k) for k in range(3)]
    plan = P.Plan(subs, panel_width=16, use_coords=False)
    plan.factor()
    p, q = _dual_vectors(plan, subs, seed=13)
    plan.apply_implicit(p, q)
    qh, ph = q.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        ref = oracle.schur(s) @ ph[o:o + s.m]
        assert np.linalg.norm(qh[o:o + s.m] - ref) <= 1e-12 * np.linalg.norm(ref), i
    plan.destroy()


def test_implicit_apply_wide_levels_match_a_sparse_solve():
    """Levels with thousands of blocks (3 x 700 independent 48 x 48
    components, three 16-column blocks each, pruned rows below the first two)
    in the one-launch-per-level sweeps; against B K^-1 B^T p from a sparse
    direct solve."""
    import scipy.sparse.linalg as spla
    _torch_init()
    subs = [_block_diagonal_subdomain(700, 48, 96, seed=41 + k) for k in range(3)]
    plan = P.Plan(subs, panel_width=16, use_coords=False)
    plan.factor()
    p, q = _dual_vectors(plan, subs, seed=17)
    plan.apply_implicit(p, q)
    qh, ph = q.cpu().numpy(), p.cpu().numpy()
    for i, s in enumerate(subs):
        o = plan.query(i)["dual_offset"]
        Bt = s.Bt_dense()
        ref = Bt.T @ spla.spsolve(s.Kreg_csr().tocsc(), Bt @ ph[o:o + s.m])
        assert np.linalg.norm(qh[o:o + s.m] - ref) <= 1e-12 * np.linalg.norm(ref), i
    plan.destroy()


def test_implicit_apply_graph_replays_match_eager():
    """The implicit apply replayed as a captured graph (use_graph) gives bit
    for bit the eager result, on repeated replays with eager work between
    them and after the output vector changes (a new capture)."""
    torch = _torch_init()
    subs = scgen.config_subdomains(2, count=3) + scgen.config_subdomains(3, count=3)
    eager = P.Plan(subs)
    eager.factor()
    p, q = _dual_vectors(eager, subs, seed=12)
    eager.apply_implicit(p, q)
    ref = q.cpu().numpy()
    eager.destroy()
    plan = P.Plan(subs, use_graph=True)
    plan.factor()
    for q2 in (torch.zeros_like(p), torch.zeros_like(p)):
        for rep in range(3):
            q2.fill_(7.0)
            junk = torch.randn(1 << 20, device="cuda")
            plan.apply_implicit(p, q2)
            junk.mul_(2.0)
            torch.cuda.synchronize()
            assert np.array_equal(q2.cpu().numpy(), ref), rep
    # alternating input and output buffers, no synchronisation in between
    ps = [p.clone(), p.clone()]
    qs = [torch.full_like(p, 7.0) for _ in range(4)]
    for k in range(4):
        plan.apply_implicit(ps[k % 2], qs[k])
    torch.cuda.synchronize()
    for k in range(4):
        assert np.array_equal(qs[k].cpu().numpy(), ref), k
    plan.destroy()


# ---------------------------------------------------------------- HIP graph

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_match_eager(precision):
    """The captured assembly, replayed several times with eager work and
    synchronisations in between, gives the eager result every time."""
    torch = _torch_init()
    subs = scgen.config_subdomains(3, count=4) + scgen.config_subdomains(1)
    eager = _assemble(subs, precision=precision)
    ref = [eager.get_F(i) for i in range(len(subs))]
    plan = P.Plan(subs, precision=precision, use_graph=True)
    plan.factor()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda")          # eager work between replays
        plan.assemble()
        junk.mul_(2.0)
        torch.cuda.synchronize()
        for i in range(len(subs)):
            assert np.array_equal(plan.get_F(i), ref[i]), (rep, i)


# ------------------------------------------------------ reach-restricted sweep

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reach_restricted_sweep_matches_full_staircase_sweep(precision):
    """Skipping the factor blocks off the elimination-tree paths of a tile's
    pivots changes nothing: F bit for bit equal to the sweep over every block
    after the first pivot, on uneven heat and elasticity subdomains, one with
    an empty interface."""
    _torch_init()
    subs = scgen.config_subdomains(2, count=10) + scgen.config_subdomains(3, count=10) + \
        scgen.config_subdomains(1)
    subs.append(subs[1].with_columns(np.zeros(0, np.int32), np.zeros(0, np.int8)))
    full = _assemble(subs, precision=precision, reach=False)
    part = _assemble(subs, precision=precision)
    for i in range(len(subs)):
        assert np.array_equal(part.get_F(i), full.get_F(i)), i
    full.destroy()
    part.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pair_merged_updates_match_separate_updates(precision):
    """The TRSM's merged updates below pairs of consecutive factor blocks
    (the default) give F bit for bit equal to one update per block
    (disable_pair_merge): a 20^3 elasticity pair of subdomains (65 pairs
    each with uniform blocks, 98 with etree blocks), uneven elasticity subdomains and scattered interior multipliers,
    with uniform and etree blocks, the staircase alone, no staircase,
    temporary-memory waves, the overlapped assembly and the pipelined
    preprocessing."""
    _torch_init()
    big = scgen.config_subdomains(5, count=2)
    assert P.host_analyze(big[0], values=False)["merge_pairs"] > 0
    subs = scgen.config_subdomains(3, count=8)
    s = scgen.box_subdomain("elasticity", (10, 10, 10), 0.1, seed=24)
    dof = np.sort(np.random.default_rng(25).choice(s.n, size=333, replace=False)).astype(np.int32)
    subs.append(s.with_columns(dof, scgen.rng.signs_from_seed(26, 333)))
    # both batches save more than the 10% of their pruned-row updates above
    # which the plan launches the merge-capable TRSM kernel
    for batch in (big, subs):
        st = [P.host_analyze(x, values=False) for x in batch]
        assert sum(h["merged_rows"] for h in st) >= 0.1 * sum(h["pruned_updates"] for h in st)
    elem = 8 if precision == "fp64" else 4
    xmax = max(x.n * 64 * ((x.m + 63) // 64) * elem for x in subs)
    cases = [(big, {}), (big, {"block_split": "etree"}), (subs, {}), (subs, {"block_split": "etree"}),
             (subs, {"reach": False}), (subs, {"staircase": False}), (subs, {"arena_cap_bytes": 2 * xmax}),
             (subs, {"assembly": "overlap"}), (subs, {"preprocess": True})]
    for batch, kw in cases:
        kw = dict(kw)
        prep = kw.pop("preprocess", False)
        plans = []
        for merge in (True, False):
            _torch_init()
            plan = P.Plan(batch, precision=precision, pair_merge=merge, **kw)
            if prep:
                plan.preprocess()
            else:
                plan.factor()
                plan.assemble()
            plans.append(plan)
        for i in range(len(batch)):
            assert np.array_equal(plans[0].get_F(i), plans[1].get_F(i)), (kw, prep, i)
        for plan in plans:
            plan.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_scattered_interior_columns(precision):
    """Multipliers on random interior DOFs (pivots spread over the whole
    elimination tree, so the visit lists and step lists have gaps everywhere)
    on a 12^3 heat subdomain and a 12^3 elasticity subdomain (n = 6591: the
    mixed SYRK takes the 128 x 128 tiles there, the FP64 SYRK the 64 x 64
    blocks), against the oracle on seeded column samples."""
    rng = np.random.default_rng(21)
    subs = []
    for kind, m in (("heat", 300), ("elasticity", 400)):
        s = scgen.box_subdomain(kind, (12, 12, 12), 1.0 / 12, seed=22)
        dof = np.sort(rng.choice(s.n, size=m, replace=False)).astype(np.int32)
        subs.append(s.with_columns(dof, scgen.rng.signs_from_seed(23, m)))
    plan = _assemble(subs, precision=precision)
    tol = TOL_FP64 if precision == "fp64" else TOL_MIXED
    for i, s in enumerate(subs):
        sel = np.sort(np.random.default_rng(i).choice(s.m, size=96, replace=False))
        F = plan.get_F(i)
        assert oracle.relF(F[np.ix_(sel, sel)], oracle.schur(s, sel=sel)) <= tol, i
    plan.destroy()


# ------------------------------------------------------ overlapped assembly

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_overlapped_assembly_matches_two_launches(precision):
    """The SYRK of one subdomain group on a second stream while the TRSM of
    the next runs gives bit for bit the F of the two-launch assembly, on a
    batch with uneven subdomains, an empty interface and more subdomains
    than XCDs and groups; repeated calls and graph replays (with eager work
    between them) agree."""
    torch = _torch_init()
    subs = (scgen.config_subdomains(2, count=40) + scgen.config_subdomains(3, count=12) +
            scgen.config_subdomains(1))
    subs.append(subs[1].with_columns(np.zeros(0, np.int32), np.zeros(0, np.int8)))
    two = _assemble(subs, precision=precision, assembly="separate")
    ref = [two.get_F(i) for i in range(len(subs))]
    for use_graph in (False, True):
        plan = P.Plan(subs, precision=precision, assembly="overlap", use_graph=use_graph)
        plan.factor()
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda")
            plan.assemble()
            junk.mul_(2.0)
            torch.cuda.synchronize()
            for i in range(len(subs)):
                assert np.array_equal(plan.get_F(i), ref[i]), (use_graph, rep, i)
        plan.destroy()


def test_overlapped_assembly_on_a_side_stream():
    """Work queued on the caller's stream after sc_assemble sees the whole F
    (the caller's stream waits for the second stream's last SYRK)."""
    torch = _torch_init()
    subs = scgen.config_subdomains(2, count=24)
    ref = _assemble(subs, assembly="separate")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = P.Plan(subs, assembly="overlap", stream=side)
        plan.factor(stream=side)
        plan.assemble(stream=side)
        st = plan.stats()
        p = torch.rand(st["dual_total"], dtype=torch.float64, device="cuda")
        q = torch.zeros_like(p)
        q_ref = torch.zeros_like(p)
        plan.apply(p, q, stream=side)
    side.synchronize()
    ref.apply(p, q_ref)
    torch.cuda.synchronize()
    assert torch.equal(q, q_ref)


def test_overlapped_assembly_is_timed_in_its_own_slot():
    _torch_init()
    subs = scgen.config_subdomains(3, count=4)
    plan = P.Plan(subs, assembly="overlap")
    plan.factor()
    plan.set_timing(True)
    plan.assemble()
    plan.assemble()
    t = plan.kernel_times()
    assert t["assemble_overlap"][1] == 2 and t["assemble_overlap"][0] > 0
    assert t["trsm"][1] == 0 and t["syrk"][1] == 0


def _median_n_star(subs, **kw):
    ns = [P.host_analyze(s, values=False, **kw)["n_star"] for s in subs]
    return ns, float(np.median(ns))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hybrid_explicit_implicit_selection(precision):
    """select_iters between the subdomains' predicted amortisation points:
    the ones with n* above it are applied with the factor, the others with
    the assembled F; sc_apply and sc_pcpg against the all-explicit plan."""
    torch = _torch_init()
    subs = scgen.config_subdomains(3, count=12)
    ns, k = _median_n_star(subs, precision=precision)
    k = int(k)
    hyb = _assemble(subs, precision=precision, select_iters=k)
    ref = _assemble(subs, precision=precision)
    imp = [hyb.selection(i)["implicit"] for i in range(len(subs))]
    assert imp == [n > k for n in ns] and any(imp) and not all(imp)
    for i in range(len(subs)):
        assert np.isclose(hyb.selection(i)["n_star"], ns[i])
        if imp[i]:
            with pytest.raises(P.ScasmError) as e:
                hyb.get_F(i)
            assert e.value.status == P.SC_ERR_STATE
        else:
            assert np.array_equal(hyb.get_F(i), ref.get_F(i))
    p, _ = _dual_vectors(hyb, subs, seed=21)
    q_h, q_r = torch.zeros_like(p), torch.zeros_like(p)
    hyb.apply(p, q_h)
    ref.apply(p, q_r)
    tol = 1e-12 if precision == "fp64" else 1e-5
    for i, s in enumerate(subs):
        o = hyb.query(i)["dual_offset"]
        a, b = q_h[o:o + s.m].cpu().numpy(), q_r[o:o + s.m].cpu().numpy()
        assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b), i
    with pytest.raises(P.ScasmError) as e:
        hyb.apply_noalloc(p, q_h)
    assert e.value.status == P.SC_ERR_UNSUPPORTED
    d = torch.from_numpy(scgen.splitmix64_uniform(77, hyb.dual_total)).cuda()
    lam_h, lam_r = torch.zeros_like(d), torch.zeros_like(d)
    hyb.pcpg(d, lam_h, 60)
    ref.pcpg(d, lam_r, 60)
    # 60 CG steps amplify the rounding differences of the two operators
    assert float(torch.linalg.norm(lam_h - lam_r) / torch.linalg.norm(lam_r)) <= (1e-6 if precision == "fp64" else 1e-4)
    hyb.destroy()
    ref.destroy()


@pytest.mark.parametrize("split", ["uniform", "etree"])
def test_all_implicit_selection_equals_the_implicit_apply(split):
    """Every subdomain selected for the implicit approach: sc_apply (the
    schedule over the listed subdomains) equals sc_apply_implicit bit for bit;
    with etree blocks both run level launches and the per-subdomain tail of
    the top levels."""
    torch = _torch_init()
    subs = scgen.config_subdomains(3, count=5) + scgen.config_subdomains(1)
    plan = _assemble(subs, select_iters=1000, select_model=(10.0, 2000.0, 1e9), block_split=split)
    assert all(plan.selection(i)["implicit"] for i in range(len(subs)))
    p, _ = _dual_vectors(plan, subs, seed=5)
    q1, q2 = torch.zeros_like(p), torch.zeros_like(p)
    plan.apply(p, q1)
    plan.apply_implicit(p, q2)
    assert torch.equal(q1, q2)
    plan.destroy()


def test_autotune_classes_tune_cache_and_plan(tmp_path):
    """Per-size-class autotuning (block split, width, SYRK work items) on
    an uneven batch; the cache file returns the same classes without timing
    again; a plan built with the classes matches the oracle."""
    _torch_init()
    subs = scgen.config_subdomains(3, count=40)
    cache = str(tmp_path / "tune.txt")
    cls = P.autotune_classes(subs, sample=2, reps=1, cache_path=cache)
    ns = np.array([s.n for s in subs])
    assert len(cls) >= 2
    assert cls[0]["n_lo"] <= ns.min() and cls[-1]["n_hi"] > ns.max()
    for a, b in zip(cls[:-1], cls[1:]):
        assert a["n_hi"] <= b["n_lo"]
    for c in cls:
        assert c["panel_width"] in (32, 48, 64) and c["block_split"] in (0, 1) and c["syrk_kind"] in (1, 2)
        assert c["ms_per_sub"] > 0
    with open(cache) as f:
        assert len([l for l in f if l.strip() and not l.startswith("#")]) == len(cls)
    again = P.autotune_classes(subs, sample=2, reps=1, cache_path=cache)
    assert [(c["n_lo"], c["n_hi"], c["panel_width"], c["block_split"], c["syrk_kind"]) for c in again] == \
        [(c["n_lo"], c["n_hi"], c["panel_width"], c["block_split"], c["syrk_kind"]) for c in cls]
    # every setting once, on a plan
    mixed_cls = [dict(c, panel_width=pw, block_split=k % 2, syrk_kind=1 + (k // 2) % 2)
                 for k, (c, pw) in enumerate(zip(cls, (32, 48, 64, 32, 48)))]
    for tc in (cls, mixed_cls):
        plan = _assemble(subs[:8], tune_classes=tc)
        _check_against_oracle(plan, subs[:8], max_full=3000)
        plan.destroy()


def test_autotune_picks_a_candidate():
    _torch_init()
    subs = scgen.config_subdomains(3, count=12)
    best, times = P.autotune(subs, candidates=(32, 64), sample=6, reps=1)
    assert best in (32, 64)
    assert all(t > 0 for t in times.values())
    assert times[best] == min(times.values())
