"""GPU parity of batched solves, graph replay and launch-shape tuning, through the C ABI.

A batch solves many independent problems with one launch per pass over the work items
of all members, replayed from a captured HIP graph.  Every member is checked against
the CPU oracle; the launch-shape choices that do not touch the arithmetic are checked
to give bitwise the same result.
"""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as WL

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-12


@pytest.fixture(scope="module")
def cs3d():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1912_03565_amd as m
    return m


DEV = "cuda:0"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle(p, dtype=np.float64):
    return O.solve(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma,
                   None, None, dtype=dtype)


def _plan_solve(cs3d, p, tuning=None):
    plan = cs3d.plan_for_problem(p, device=DEV)
    if tuning:
        plan.set_tuning(tuning)
    u = plan.solve(p.f.to(DEV)).cpu().numpy()[0]
    plan.close()
    return u


def _batch(cs3d, probs):
    return cs3d.Batch([cs3d.batch_member(p) for p in probs], device=DEV)


# members covering every transform path of the general kernel variant: dense sine sums,
# FFT lengths 64 ... 1024, single planes, ragged tiles, every scheme
MIXED = [("helm6", 30, 17, 9), ("cd4", 100, 63, 12), ("helm4", 511, 63, 6), ("helm4", 63, 1023, 4),
         ("helm2", 5, 7, 6), ("cd4", 3, 2, 1), ("helm6", 63, 127, 33), ("helm4", 127, 63, 20)]


def test_batch_general_variant_matches_oracle(cs3d):
    probs = [WL.noise_problem(nx, ny, nz, s, seed=500 + i, boundary=False)
             for i, (s, nx, ny, nz) in enumerate(MIXED)]
    print("batch of", [p.name for p in probs], flush=True)
    b = _batch(cs3d, probs)
    us = b.solve([p.f[0].to(DEV) for p in probs])
    st = b.stats()
    assert st["bad_pivots"] == 0
    for i, (p, u) in enumerate(zip(probs, us)):
        ref = _oracle(p, np.longdouble)
        u64 = _oracle(p).U
        bar = max(TOL_FP64, 4.0 * _rel(u64, ref.U))
        err = _rel(u.cpu().numpy(), ref.U)
        ms = b.member_stats(i)
        print(f"  {p.name}: rel err {err:.3e} (bar {bar:.1e}) minpiv {ms['min_abs_pivot']:.3e}", flush=True)
        assert err < bar
        assert abs(ms["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)
        # the same per-item code as a plan of this member
        assert _rel(u.cpu().numpy(), _plan_solve(cs3d, p)) < 1e-14
    b.close()


def _weight_sensitivity(p, dtype):
    """Relative change of the solution when every stencil weight moves by one FP64 unit in
    the last place (random sign): the spread that FP64 rounding of the weights of Sections
    3.3-3.5 alone causes on this member."""
    W = O.stencil_weights(p.scheme, p.nz, p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma)
    F = O.rhs(p.scheme, p.f[0].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.gamma)
    ref = O.solve(None, None, p.hx, p.hy, p.hz, W=W, F=F, dtype=dtype).U
    rng = np.random.default_rng(1)
    Wp = W * (1.0 + np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=W.shape))
    return _rel(O.solve(None, None, p.hx, p.hy, p.hz, W=Wp, F=F, dtype=dtype).U, ref)


def test_batch_of_64_uneven_problems(cs3d):
    """64 problems, per-axis sizes drawn from {63, 127, 255}, HELM4/HELM6/CD4 in turn with
    k0 ~ U[5, 60] or gamma ~ U[-100, -5], solved in one batch.

    * every member against a plan of its own (the same per-item code): 1e-14;
    * the six smallest members against the extended-precision oracle, and every eighth
      member against the FP64 oracle.  The bar is 1e-12, or, on an indefinite member with
      small pivots, four times what FP64 rounding alone moves its result: the change under
      one-ulp perturbations of the stencil weights (and, against the extended-precision
      oracle, the FP64 oracle's own error)."""
    probs = WL.batch_members(seed=104, count=64, sizes=(63, 127, 255))
    b = _batch(cs3d, probs)
    fs = [p.f[0].to(DEV) for p in probs]
    us = b.solve(fs)
    st = b.stats()
    print(f"batch of 64: {sum(p.nx * p.ny * p.nz for p in probs)} unknowns, "
          f"min pivot {st['min_abs_pivot']:.3e}", flush=True)
    assert st["bad_pivots"] == 0 and st["status"] == 0
    bitwise = 0
    for p, u in zip(probs, us):
        up = _plan_solve(cs3d, p)
        ug = u.cpu().numpy()
        assert _rel(ug, up) < 1e-14, p.name
        bitwise += int(np.array_equal(ug, up))
    print(f"  {bitwise} of 64 members bitwise equal to their plan's solve", flush=True)
    vols = [p.nx * p.ny * p.nz for p in probs]
    small = np.argsort(vols)[:6].tolist()
    for i in sorted(set(small) | set(range(0, 64, 8))):
        p, ug = probs[i], us[i].cpu().numpy()
        if i in small:
            ref = _oracle(p, np.longdouble).U
            bar = max(TOL_FP64, 4.0 * _rel(_oracle(p).U, ref))
            kind = "extended"
        else:
            ref = _oracle(p).U
            bar, kind = TOL_FP64, "FP64"
        err = _rel(ug, ref)
        if err >= bar:
            bar = max(bar, 4.0 * _weight_sensitivity(p, np.longdouble if i in small else np.float64))
        print(f"  {p.name}: vs {kind} oracle {err:.3e} (bar {bar:.1e})", flush=True)
        assert err < bar, (p.name, err, bar)
    b.close()


def test_graph_replay_and_pointer_changes(cs3d):
    """Replays of the captured graph, with eager work in between, give bitwise the result of
    pass-by-pass launches; new input/output tensors are picked up (descriptor upload) and a
    right-hand side scaled by 2 gives exactly twice the solution."""
    probs = [WL.noise_problem(nx, ny, nz, s, seed=900 + i, boundary=False)
             for i, (s, nx, ny, nz) in enumerate([("helm6", 63, 63, 31), ("cd4", 127, 63, 17),
                                                  ("helm4", 255, 127, 9)])]
    b = _batch(cs3d, probs)
    fs = [p.f[0].to(DEV) for p in probs]
    b.set_tuning({"graph": 0})
    ref = [u.clone() for u in b.solve(fs)]
    st = b.stats()
    assert len(st["stage_ms"]) == 5 and all(t > 0 for t in st["stage_ms"])
    b.set_tuning({"graph": 1})
    us = b.outputs()
    for k in range(3):
        b.solve(fs, us)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device=DEV).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for u, r in zip(us, ref):
            assert torch.equal(u, r), f"replay {k}"
    assert b.stats()["stage_ms"] == []
    fs2 = [2.0 * f for f in fs]
    us2 = b.solve(fs2)
    for u, r in zip(us2, ref):
        assert torch.equal(u, 2.0 * r)
    b.close()


def test_batch_tuning_is_bitwise_neutral(cs3d):
    probs = [WL.noise_problem(nx, ny, nz, s, seed=700 + i, boundary=False)
             for i, (s, nx, ny, nz) in enumerate([("helm4", 63, 255, 70), ("helm6", 127, 63, 45)])]
    b = _batch(cs3d, probs)
    fs = [p.f[0].to(DEV) for p in probs]
    ref = [u.clone() for u in b.solve(fs)]
    for t in ({"zchunk": 8, "order": 0}, {"zchunk": 64, "order": 1, "graph": 0}, {"zchunk": 512}):
        b.set_tuning(t)
        for u, r in zip(b.solve(fs), ref):
            assert torch.equal(u, r), t
    best, ms = b.autotune(fs, reps=1)
    assert best["graph"] == 1 and best["zchunk"] in (16, 32, 64, 128) and ms > 0
    for u, r in zip(b.solve(fs), ref):
        assert torch.equal(u, r)
    b.close()


def test_plan_tuning_choices(cs3d):
    """zchunk and xpersist leave the result bitwise unchanged; ywpl (another radix split
    of the 1024-point y transform) stays within the FP64 parity bar."""
    p = WL.noise_problem(63, 1023, 6, "helm4", seed=321, boundary=False)
    plan = cs3d.plan_for_problem(p, device=DEV)
    f = p.f.to(DEV)
    base = plan.solve(f).clone()
    assert plan.tuning()["ywpl"] == 2
    for t in ({"zchunk": 8}, {"zchunk": 512}, {"xpersist": 0}, {"zchunk": 16, "xpersist": 1}):
        plan.set_tuning(t)
        assert torch.equal(plan.solve(f), base), t
    plan.set_tuning({"ywpl": 1, "zchunk": 32})
    u1 = plan.solve(f).cpu().numpy()
    ref = _oracle(p, np.longdouble).U
    assert _rel(u1[0], ref) < TOL_FP64
    assert _rel(base.cpu().numpy()[0], ref) < TOL_FP64
    best, ms = plan.autotune(f, reps=1)
    assert best["ywpl"] in (1, 2) and best["zchunk"] in (16, 32, 64, 128) and ms > 0
    plan.close()


def test_tuning_cache_roundtrip(cs3d, tmp_path, monkeypatch):
    monkeypatch.setenv("CS3D_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setenv("CS3D_AUTOTUNE", "1")
    p = WL.noise_problem(63, 63, 20, "helm6", seed=11, boundary=False)
    plan = cs3d.plan_for_problem(p, device=DEV)
    f = p.f.to(DEV)
    t1 = cs3d.tuned_plan(plan, f, reps=1)
    plan2 = cs3d.plan_for_problem(p, device=DEV)
    t2 = cs3d.tuned_plan(plan2, f, reps=1)  # a cache hit: no tuning run
    assert t1 == t2 == plan2.tuning()
    plan.close()
    plan2.close()


def test_singular_modes_are_reported(cs3d):
    """A stencil whose modal eigenvalues all vanish (zero weights): every pivot of the LU is
    zero, the solve completes and cs3d_get_stats reports E_SINGULAR with the count."""
    nx, ny, nz = 63, 5, 3
    W = np.zeros((nz, 3, 4))
    plan = cs3d.Plan(nx, ny, nz, 1.0, 1.0, 1.0, "weights", weights=W, device=DEV)
    F = torch.ones((1, nz, ny, nx), dtype=torch.float64, device=DEV)
    plan.solve_assembled(F)
    st = plan.stats()
    assert st["status"] == cs3d.native.E_SINGULAR
    assert st["bad_pivots"] == nx * ny * nz
    with pytest.raises(cs3d.CS3DError):
        plan.stats(raise_singular=True)
    plan.close()


def test_workspace_errors(cs3d):
    import ctypes
    N = cs3d.native
    p = WL.noise_problem(63, 63, 8, "helm4", seed=5, boundary=False)
    plan = cs3d.plan_for_problem(p, device=DEV)
    small = torch.empty(1024, dtype=torch.uint8, device=DEV)
    ptr = small.data_ptr() + ((-small.data_ptr()) % 256)
    assert N.lib.cs3d_set_workspace(plan._plan, ptr + 1, 512) == N.E_INVAL  # misaligned
    assert N.lib.cs3d_set_workspace(plan._plan, ptr, 512) == N.OK
    f = p.f.to(DEV)
    u = torch.empty((1, 8, 63, 63), dtype=torch.float64, device=DEV)
    st = N.lib.cs3d_solve(plan._plan, 1, f.data_ptr(), None, None, u.data_ptr(), ctypes.c_void_p(0))
    assert st == N.E_WORKSPACE
    assert N.lib.cs3d_solve(plan._plan, 2, f.data_ptr(), None, None, u.data_ptr(), ctypes.c_void_p(0)) == N.E_INVAL
    plan.close()


def test_rhs_sharing_in_y_passes(cs3d):
    """Right-hand sides sharing a y-pass workgroup (1, 2 or 4 of them, with a ragged last
    group of five) give bitwise the same solution, which matches the oracle per right-hand
    side; the pivot statistics count each modal pivot once."""
    p = WL.noise_problem(127, 63, 21, "helm6", seed=4242, nrhs=5)
    plan = cs3d.plan_for_problem(p, device=DEV)
    f, gl, gh = p.f.to(DEV), p.g_lo.to(DEV), p.g_hi.to(DEV)
    outs = {}
    for nr in (1, 2, 4):
        plan.set_tuning({"yrhs": nr})
        outs[nr] = plan.solve(f, gl, gh).clone()
        st = plan.stats()
        assert st["bad_pivots"] == 0
    assert torch.equal(outs[1], outs[2]) and torch.equal(outs[1], outs[4])
    for r in (0, 3, 4):
        ref = O.solve(p.scheme, p.f[r].numpy(), p.hx, p.hy, p.hz, p.k2, p.k2_z, p.k2_zz, p.gamma,
                      p.g_lo[r].numpy(), p.g_hi[r].numpy(), dtype=np.longdouble)
        assert _rel(outs[4][r].cpu().numpy(), ref.U) < TOL_FP64
        assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)
    plan.close()
