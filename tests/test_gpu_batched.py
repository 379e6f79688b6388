"""GPU parity of the batched solver (many chromosome blocks stepped together).

Each problem of a batch must agree with the FP64 oracle run on that problem
alone -- singular values to 1e-10 relative, singular vectors to 1e-6 where the
relative gap to the neighbours exceeds 1e-2 -- whatever the other problems of
the batch do.  The steps replayed from the captured HIP graph must reproduce
the eagerly launched kernels exactly (the kernels sum in fixed orders), and
repeated solves must agree bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth   # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_1808_03374_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def chromosome_batch(n, chroms, scale):
    """The 22-block genome recipe at n individuals, block sizes divided by `scale`."""
    sizes = synth.chromosome_sizes()
    gs = [synth.config("c4", n=n, p=max(64, sizes[c - 1] // scale), chrom=c) for c in chroms]
    return gs, [dev(g.packed) for g in gs]


def start_vectors(gs):
    return [synth.start_vector(g.p, 100 + q) for q, g in enumerate(gs)]


def oracle_solutions(gs, k, v0s):
    out = []
    for g, v0 in zip(gs, v0s):
        op = oracle.PackedOperator(g.packed, g.n, g.p)
        out.append((op, oracle.gkl_svd(op, k, tol=1e-12, v0=v0)))
    return out


def check_against_oracle(sig, U, V, op, ref, k):
    sig = sig.cpu().numpy()
    U = U.cpu().numpy()
    V = V.cpu().numpy()
    assert np.all(np.abs(sig - ref.sigma) <= 1e-10 * ref.sigma), np.abs(sig - ref.sigma) / ref.sigma
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-8
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-8
    r1, r2, _ = oracle.certificate(op, sig, U, V)
    assert max(r1.max(), r2.max()) <= 1e-9 * sig[0]
    gap = np.abs(np.diff(ref.sigma)) / ref.sigma[:-1]
    for i in range(k - 1):
        if gap[i] > 1e-2 and (i == 0 or gap[i - 1] > 1e-2):
            assert oracle.subspace_angles(V[:, i:i + 1], ref.V[:, i:i + 1]).max() < 1e-6
            assert oracle.subspace_angles(U[:, i:i + 1], ref.U[:, i:i + 1]).max() < 1e-6


def run_batch(gk, Gs, gs, k, v0s, **opts):
    v0 = dev(np.concatenate(v0s))
    ctx = gk.BatchedContext(Gs, [g.n for g in gs], [g.p for g in gs], k, tol=1e-11,
                            reorth=gk.GKL_REORTH_FULL, v0=v0, **opts)
    try:
        sig, Us, Vs, st, infos = ctx.solve()
        plan = ctx.plan()
    finally:
        ctx.close()
    return sig, Us, Vs, st, infos, plan


def fmt_option(gk, fmt):
    # A^T u from the tables, or in int8 limbs (A v is always from the tables)
    return gk.GKL_FP64_LUT if fmt == "lut" else gk.GKL_FP64_LUT_LIMBS


@pytest.mark.parametrize("fmt", ["lut", "limbs"])
@pytest.mark.parametrize("krylov", [0, 16])
def test_batched_matches_oracle_per_problem(gk, krylov, fmt):
    # six blocks of the 4-subpopulation genome, 700 individuals, 96..2,000 SNPs
    gs, Gs = chromosome_batch(700, [1, 4, 9, 14, 19, 22], 40)
    k = 5
    v0s = start_vectors(gs)
    refs = oracle_solutions(gs, k, v0s)
    sig, Us, Vs, st, infos, _ = run_batch(gk, Gs, gs, k, v0s, krylov_dim=krylov,
                                          fp64_products=fmt_option(gk, fmt))
    assert st == gk.GKL_OK
    assert all(i.fp64_products == fmt_option(gk, fmt) for i in infos)
    for q, (op, ref) in enumerate(refs):
        assert infos[q].converged == 1
        check_against_oracle(sig[q], Us[q], Vs[q], op, ref, k)
    if krylov:
        assert max(i.restarts for i in infos) >= 1


@pytest.mark.parametrize("fmt", ["lut", "limbs"])
def test_graph_replay_matches_eager_launches(gk, fmt):
    gs, Gs = chromosome_batch(640, [2, 7, 12, 21], 30)
    k = 4
    v0s = start_vectors(gs)
    f = fmt_option(gk, fmt)
    a = run_batch(gk, Gs, gs, k, v0s, krylov_dim=14, graph=1, fp64_products=f)
    # eager work on the same stream between the two solves
    x = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    float((x * x).sum())
    b = run_batch(gk, Gs, gs, k, v0s, krylov_dim=14, graph=0, fp64_products=f)
    c = run_batch(gk, Gs, gs, k, v0s, krylov_dim=14, graph=1, fp64_products=f)
    for q in range(len(gs)):
        for r in (b, c):
            assert torch.equal(a[0][q], r[0][q])
            assert torch.equal(a[1][q], r[1][q])
            assert torch.equal(a[2][q], r[2][q])
        assert a[4][q].steps == b[4][q].steps == c[4][q].steps


def test_problems_converge_and_leave_independently(gk):
    # one small well-separated problem next to larger ones: it stops early and
    # the others are unaffected
    gs, Gs = chromosome_batch(600, [1, 22, 3], 20)
    k = 3
    v0s = start_vectors(gs)
    refs = oracle_solutions(gs, k, v0s)
    sig, Us, Vs, st, infos, _ = run_batch(gk, Gs, gs, k, v0s, check_every=2)
    assert st == gk.GKL_OK
    assert len({i.steps for i in infos}) >= 2
    for q, (op, ref) in enumerate(refs):
        check_against_oracle(sig[q], Us[q], Vs[q], op, ref, k)


@pytest.mark.parametrize("fmt", ["lut", "limbs"])
def test_autotuned_geometry(gk, fmt):
    gs, Gs = chromosome_batch(900, [3, 8, 17], 25)
    k = 4
    v0s = start_vectors(gs)
    f = fmt_option(gk, fmt)
    a = run_batch(gk, Gs, gs, k, v0s, krylov_dim=16, fp64_products=f)
    b = run_batch(gk, Gs, gs, k, v0s, krylov_dim=16, autotune=1, fp64_products=f)
    plan = b[5]
    assert plan["mv_target"] in (192, 384, 768, 1536)
    assert plan["rmv_target"] in (192, 384, 768, 1536)
    assert plan["grid_mv"] in (512, 1024, 2048) and plan["grid_rmv"] in (512, 1024, 2048)
    assert plan["mv_ms"] > 0 and plan["rmv_ms"] > 0
    for q in range(len(gs)):
        s0, s1 = a[0][q].cpu().numpy(), b[0][q].cpu().numpy()
        assert np.all(np.abs(s0 - s1) <= 1e-10 * s0)


@pytest.mark.parametrize("fmt", ["lut", "limbs"])
def test_problems_of_different_sizes_and_a_single_problem(gk, fmt):
    # individuals differ between problems too; and a batch of one
    sizes = [(300, 1500, 5), (900, 700, 9), (520, 2600, 13)]
    gs = [synth.config("c4", n=n, p=p, chrom=c) for n, p, c in sizes]
    Gs = [dev(g.packed) for g in gs]
    k = 4
    v0s = start_vectors(gs)
    refs = oracle_solutions(gs, k, v0s)
    f = fmt_option(gk, fmt)
    sig, Us, Vs, st, infos, _ = run_batch(gk, Gs, gs, k, v0s, krylov_dim=16, fp64_products=f)
    assert st == gk.GKL_OK
    for q, (op, ref) in enumerate(refs):
        check_against_oracle(sig[q], Us[q], Vs[q], op, ref, k)
    sig1, Us1, Vs1, st1, _, _ = run_batch(gk, Gs[1:2], gs[1:2], k, v0s[1:2], krylov_dim=16,
                                          fp64_products=f)
    assert st1 == gk.GKL_OK
    check_against_oracle(sig1[0], Us1[0], Vs1[0], refs[1][0], refs[1][1], k)


def test_rank_deficient_problem_reports_breakdown(gk):
    # a two-group matrix has rank one: asking for three triplets breaks the
    # Lanczos recurrence on that problem; the other problem still converges
    n, p = 40, 30
    codes = np.zeros((n, p), dtype=np.int64)
    codes[n // 2:] = 2
    g0 = synth.Genotypes(synth.pack_codes(codes), n, p, (n + 3) // 4, {})
    g1 = synth.config("c4", n=300, p=900, chrom=4)
    gs = [g0, g1]
    Gs = [dev(g.packed) for g in gs]
    k = 3
    v0s = start_vectors(gs)
    v0 = dev(np.concatenate(v0s))
    ctx = gk.BatchedContext(Gs, [g.n for g in gs], [g.p for g in gs], k, tol=1e-11,
                            reorth=gk.GKL_REORTH_FULL, v0=v0)
    SA = [torch.empty(k, dtype=torch.float64, device="cuda") for _ in gs]
    UA = [torch.empty((k, g.n), dtype=torch.float64, device="cuda") for g in gs]
    VA = [torch.empty((k, g.p), dtype=torch.float64, device="cuda") for g in gs]
    infos = (gk.gkl_info * 2)()
    import ctypes
    arr = lambda xs: (ctypes.c_void_p * 2)(*[x.data_ptr() for x in xs])
    st = gk.lib.gkl_solve_batched(ctypes.c_void_p(ctx.ctx), arr(SA), arr(UA),
                                  (ctypes.c_int64 * 2)(*[g.n for g in gs]), arr(VA),
                                  (ctypes.c_int64 * 2)(*[g.p for g in gs]), infos)
    assert st == gk.GKL_ERR_BREAKDOWN
    assert "broke down" in gk.gkl_last_error(ctx.ctx)
    assert infos[0].converged == 0 and infos[1].converged == 1
    op, ref = oracle_solutions([g1], k, v0s[1:])[0]
    check_against_oracle(SA[1], UA[1].T, VA[1].T, op, ref, k)
    ctx.close()
