"""GPU parity of batched solves, graph replay and launch-shape tuning, through the C ABI.

A batch solves many independent problems with one launch per pass over the work items
of all members, replayed from a captured HIP graph.  Every member is checked against
the extended-precision CPU oracle, element by element and in the 2-norm, with the bar of
the plan path fixed from the oracle alone (``parity.py``); the launch-shape choices that
do not touch the arithmetic are checked to give bitwise the same result.
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle_pool
import parity as PT
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


def _kw(p):
    return dict(scheme=p.scheme, f=p.f[0].numpy(), hx=p.hx, hy=p.hy, hz=p.hz, k2=p.k2, k2_z=p.k2_z,
                k2_zz=p.k2_zz, gamma=p.gamma)


def _check_members(probs, us, label):
    """Every member against the extended-precision oracle (CPU worker processes); the bar of
    each is 1e-12, or four times the FP64 noise floor of that member (parity.Bar.from_errors:
    the FP64 oracle's error and the one-ulp weight and eigenvalue sensitivities), per norm,
    from the oracle alone."""
    res = oracle_pool.extended_comparisons([(p.name, _kw(p), u.cpu().numpy()) for p, u in zip(probs, us)])
    worst = 0.0
    for p, r in zip(probs, res):
        bar = PT.Bar.from_errors(r["fp64_oracle"], list(r["sensitivity"].values()))
        l2, mx = r["hip"]
        print(f"  {p.name}: rel L2 {l2:.3e} (bar {bar.l2:.1e}), rel max {mx:.3e} (bar {bar.mx:.1e})"
              + (f"{bar.why}, min pivot {r['minpiv']:.2e}" if bar.why else ""), flush=True)
        assert l2 < bar.l2 and mx < bar.mx, (label, p.name, l2, mx, bar.l2, bar.mx)
        worst = max(worst, l2 / bar.l2, mx / bar.mx)
    print(f"  {label}: {len(probs)} members, largest error / bar {worst:.2f}", flush=True)
    return res


def test_batch_general_variant_matches_oracle(cs3d):
    probs = [WL.noise_problem(nx, ny, nz, s, seed=500 + i, boundary=False)
             for i, (s, nx, ny, nz) in enumerate(MIXED)]
    print("batch of", [p.name for p in probs], flush=True)
    b = _batch(cs3d, probs)
    us = b.solve([p.f[0].to(DEV) for p in probs])
    st = b.stats()
    assert st["bad_pivots"] == 0
    res = _check_members(probs, us, "general variant")
    for i, (p, u, r) in enumerate(zip(probs, us, res)):
        ms = b.member_stats(i)
        assert abs(ms["min_abs_pivot"] - r["minpiv"]) <= 1e-9 * max(1.0, r["minpiv"])
        # the same per-item code as a plan of this member
        PT.check(f"{p.name} batch vs own plan", u.cpu().numpy(), _plan_solve(cs3d, p), PT.Bar.fixed(1e-14))
    b.close()


@pytest.mark.timeout(900)  # host oracle work in worker processes
def test_batch_of_64_uneven_problems(cs3d):
    """64 problems, per-axis sizes drawn from {63, 127, 255}, HELM4/HELM6/CD4 in turn with
    k0 ~ U[5, 60] or gamma ~ U[-100, -5], solved in one batch.

    * every member against the extended-precision oracle (about a minute of host work in
      worker processes), element by element and in the 2-norm, with the bar of the plan
      path: 1e-12, or four times the FP64 oracle's own error on an indefinite member with
      small pivots (printed with the numbers);
    * every member against a plan of its own (the same per-item code): 1e-14."""
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
        l2, mx = PT.errors(ug, up)
        assert l2 < 1e-14 and mx < 1e-14, (p.name, l2, mx)
        bitwise += int(np.array_equal(ug, up))
    print(f"  {bitwise} of 64 members bitwise equal to their plan's solve", flush=True)
    b.close()
    _check_members(probs, us, "64-member batch")


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
    b.set_tuning({"pack": 0})  # (packed lines run other kernels: test_packed_lines_*)
    for u, r in zip(b.solve(fs), ref):
        assert torch.equal(u, r)
    b.close()


# Packed lines (tuning "pack"): x-pass tiles of 32 (64-point) or 16 (128-point) lines, some
# reaching past the row length (ldy 16 and 48 against 32-line tiles); y-pass groups of 16
# or 8 lines whose last group leaves part of a wave inactive (N_x = 37, 99)
PACKED_GENERAL = [("helm6", 63, 63, 31), ("helm4", 63, 15, 9), ("helm6", 63, 47, 8), ("cd4", 127, 47, 12),
                  ("helm4", 37, 63, 10), ("cd4", 99, 127, 12), ("helm2", 127, 79, 7), ("helm4", 255, 63, 5)]
PACKED_DEFAULT = [("helm6", 63, 63, 31), ("helm4", 127, 255, 20), ("cd4", 255, 63, 9), ("helm6", 63, 127, 17)]


@pytest.mark.parametrize("members", [PACKED_GENERAL, PACKED_DEFAULT], ids=["general", "default"])
def test_packed_lines_match_unpacked_and_oracle(cs3d, members):
    """A wave carrying 4 lines of a 64-point or 2 of a 128-point transform (batch tuning
    pack = 1) runs the same arithmetic per line as one line per wave, compiled into other
    kernels: the results agree to rounding (relative 1e-14 element by element), in eager
    launches and in graph replays (each replay bitwise equal to the first packed solve),
    with the same pivot statistics; every member also against the oracle."""
    probs = [WL.noise_problem(nx, ny, nz, s, seed=1300 + i, boundary=False)
             for i, (s, nx, ny, nz) in enumerate(members)]
    print("batch of", [p.name for p in probs], flush=True)
    b = _batch(cs3d, probs)
    fs = [p.f[0].to(DEV) for p in probs]
    b.set_tuning({"pack": 0, "graph": 0})
    ref = [u.clone() for u in b.solve(fs)]
    piv0 = [b.member_stats(i)["min_abs_pivot"] for i in range(len(probs))]
    packed = None
    for graph in (0, 1):
        b.set_tuning({"pack": 1, "graph": graph})
        assert b.tuning()["pack"] == 1
        for rep in range(2):
            us = b.solve(fs)
            if packed is None:
                packed = [u.clone() for u in us]
                for p, u, r in zip(probs, us, ref):
                    d = (u - r).abs().max().item() / max(r.abs().max().item(), 1e-300)
                    print(f"  {p.name}: packed vs unpacked max rel diff {d:.2e}"
                          f"{' (bitwise)' if torch.equal(u, r) else ''}", flush=True)
                    assert d < 1e-14, (p.name, d)
            for p, u, r in zip(probs, us, packed):
                assert torch.equal(u, r), (p.name, graph, rep)
        assert b.stats()["bad_pivots"] == 0
        piv = [b.member_stats(i)["min_abs_pivot"] for i in range(len(probs))]
        assert all(abs(a - c) <= 1e-12 * c for a, c in zip(piv, piv0)), (piv, piv0)
    _check_members(probs, us, "packed lines")
    best, ms = b.autotune(fs, reps=1)
    assert best["pack"] in (0, 1) and best["graph"] == 1 and ms > 0
    print(f"  autotune: pack {best['pack']}, {ms:.3f} ms per solve", flush=True)
    for u, r in zip(b.solve(fs), packed if best["pack"] else ref):
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
    bar = PT.oracle_bar(_kw(p), ref)
    PT.check("one wave per 1024-point y line", u1[0], ref, bar)
    PT.check("two waves per 1024-point y line", base.cpu().numpy()[0], ref, bar)
    best, ms = plan.autotune(f, reps=1)
    assert best["ywpl"] in (1, 2) and best["zchunk"] in (16, 32, 64, 128) and ms > 0
    plan.close()


@pytest.mark.parametrize("nx,ny,nz", [(511, 63, 6), (1023, 31, 4)])
def test_x_pass_tile_pairs_persistent_or_not(cs3d, nx, ny, nz):
    """x lines of 512 and 1024 points: the forward x pass takes its tiles in pairs (the two
    halves of the lines of G).  A resident grid walking the pairs and one workgroup per pair
    give bitwise the same solution, which matches the oracle."""
    p = WL.noise_problem(nx, ny, nz, "helm4", seed=4100 + nx, boundary=False)
    plan = cs3d.plan_for_problem(p, device=DEV)
    f = p.f.to(DEV)
    plan.set_tuning({"xpersist": 1})
    base = plan.solve(f).clone()
    plan.set_tuning({"xpersist": 0})
    assert torch.equal(plan.solve(f), base)
    ref = _oracle(p, np.longdouble).U
    PT.check(f"{p.name} tile pairs", base.cpu().numpy()[0], ref, PT.oracle_bar(_kw(p), ref))
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
        kw = dict(scheme=p.scheme, f=p.f[r].numpy(), hx=p.hx, hy=p.hy, hz=p.hz, k2=p.k2, k2_z=p.k2_z,
                  k2_zz=p.k2_zz, gamma=p.gamma, g_lo=p.g_lo[r].numpy(), g_hi=p.g_hi[r].numpy())
        ref, _ = PT.oracle_pair(kw)
        PT.check(f"rhs {r}, four per y workgroup", outs[4][r].cpu().numpy(), ref.U, PT.oracle_bar(kw, ref.U))
        assert abs(st["min_abs_pivot"] - ref.minpiv) <= 1e-9 * max(1.0, ref.minpiv)
    plan.close()
