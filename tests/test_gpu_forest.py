"""Batched scenes (a forest) on the GPU.

Every scene of a forest is computed by the same per-bucket kernels as a lone
tree, only launched over the work items of all scenes at once, so:

  * each scene's J equals that of its own tree's single-scene call to FP32
    rounding of the atomic sums (checked to 1e-5 relative with the usual
    floor), and the oracle's to the J tolerance 1e-4;
  * the batched adjoint equals each scene's single-scene adjoint to the
    gradient tolerance of the adjoint tests, and passes a dot-product test
    against the oracle's forward-mode derivative;
  * a HIP graph captured from the batched calls replays to the eager result,
    also with different active flags written into the same buffer between
    replays (individual time steps).
"""
import numpy as np
import pytest

import oracle
from paper_2310_15235_amd import scenes

pytestmark = pytest.mark.gpu

J_TOL = 1e-4
SAME_TOL = 1e-5


def _api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_15235_amd import api
    return api


def _rel(a, b):
    floor = 1e-12 * np.abs(b).max(axis=-1, keepdims=True)
    return np.abs(a - b) / np.maximum(np.abs(b), np.maximum(floor, 1e-300))


def mixed_scenes():
    """Six small scenes covering the per-scene parameters: band counts 1-4,
    N_side 1, 2 and 4, uniform and log-normal media, a background, the thick
    factor off, and a one-bucket scene."""
    bg4 = np.array([0.3, 0.2, 0.1, 0.05], np.float32)
    return [
        scenes.uniform_scene(n=3000, seed=11, n_src=40, bands=(1.0,), nside=1),
        scenes.lognormal_scene(n=5000, seed=12, grid=16, bands=(1.0, 10.0, 100.0), nside=2),
        scenes.uniform_scene(n=2048, seed=13, n_src=32, bands=(1.0, 10.0), nside=4),
        scenes.lognormal_scene(n=2500, seed=14, grid=16, bands=(1.0, 10.0, 100.0, 1000.0),
                               nside=2, background=True, bg=bg4),
        scenes.uniform_scene(n=900, seed=15, n_src=12, bands=(2.0,), nside=2, thick_corr=False),
        scenes.uniform_scene(n=7, seed=16, n_src=2, bands=(1.0, 10.0), nside=1),
    ]


def _actives(scs, frac, seed):
    return [np.ones(s.n, np.uint8) if frac >= 1.0 else scenes.active_subset(s, frac, seed + i)
            for i, s in enumerate(scs)]


def _single_J(api, F, s, sc, act):
    import torch
    T = F.scene_tree(s)
    a = torch.as_tensor(act, device="cuda")
    bg = None
    if sc.background:
        bg = torch.as_tensor(np.asarray(sc.bg, np.float32), device="cuda")
    J = T.compute_J(a, bg).cpu().numpy()
    T.check()
    return J


@pytest.mark.parametrize("frac", [1.0, 0.1])
def test_forest_J_matches_single_trees_and_oracle(frac):
    api = _api()
    scs = mixed_scenes()
    F = api.Forest(scs)
    acts = _actives(scs, frac, seed=50)
    Jf = F.compute_J(F.flat_active(acts))
    F.check()
    parts = [p.cpu().numpy() for p in F.split(Jf)]
    for s, (sc, act) in enumerate(zip(scs, acts)):
        m = act.astype(bool)
        assert np.all(parts[s][:, ~m] == 0.0)
        Js = _single_J(api, F, s, sc, act)
        assert np.max(_rel(parts[s][:, m], Js[:, m])) <= SAME_TOL, sc.name
        Jo, co = oracle.OracleTree(sc).compute_J(act)
        assert np.max(_rel(parts[s][:, m], Jo[:, m])) <= J_TOL, sc.name
        cg = F.counters(s)
        for k in ("buckets", "segments", "source_entries", "absorber_entries"):
            assert cg[k] == co[k], (sc.name, k, cg[k], co[k])
    tot = F.counters(-1)
    assert tot["buckets"] == sum(F.counters(s)["buckets"] for s in range(F.S))
    F.close()


def test_forest_graph_replay_with_changing_active_sets():
    api = _api()
    import torch
    scs = mixed_scenes()
    F = api.Forest(scs)
    act_buf = F.flat_active(_actives(scs, 1.0, 0))
    J = F.new_J()
    F.compute_J(act_buf, out=J)          # eager warm-up (kernel tables, occupancy)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        F.compute_J(act_buf, out=J)
    for rep, frac in enumerate([1.0, 0.3, 0.05, 1.0]):
        acts = _actives(scs, frac, seed=100 + rep)
        act_buf.copy_(F.flat_active(acts))
        J.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = J.cpu().numpy()
        ref = F.compute_J(act_buf).cpu().numpy()
        F.check()
        # same kernels, same inputs: equal to FP32 rounding of the atomic sums
        assert np.max(_rel(got, ref)) <= SAME_TOL, (rep, frac)
        m = F.flat_active(acts).cpu().numpy().astype(bool)
        for s, p in enumerate(F.split(torch.as_tensor(got))):
            ms = m[F.offsets[s]:F.offsets[s + 1]]
            assert np.all(p.numpy()[:, ~ms] == 0.0)
    F.close()


def test_forest_full_batched_workload_matches_single_trees():
    """The 64-scene workload (log-uniform 2^12..2^17 elements, 1-4 bands,
    N_side 1/2/4, uniform and log-normal media) with per-scene active
    fractions of 1%, 10% and 100%: every scene against its own tree."""
    api = _api()
    scs = scenes.batched_scenes(64)
    F = api.Forest(scs)
    rng = np.random.default_rng(7)
    fracs = rng.choice([0.01, 0.1, 1.0], size=len(scs))
    acts = [scenes.active_subset(s, f, 200 + i) if f < 1.0 else np.ones(s.n, np.uint8)
            for i, (s, f) in enumerate(zip(scs, fracs))]
    parts = [p.cpu().numpy() for p in F.split(F.compute_J(F.flat_active(acts)))]
    F.check()
    for s, (sc, act) in enumerate(zip(scs, acts)):
        m = act.astype(bool)
        Js = _single_J(api, F, s, sc, act)
        assert np.max(_rel(parts[s][:, m], Js[:, m])) <= SAME_TOL, sc.name
    F.close()


def _close(got, ref, rtol):
    tol = rtol * np.abs(ref) + 1e-6 * np.abs(ref).max()
    assert np.all(np.abs(got - ref) <= tol), float(np.max(np.abs(got - ref) - tol))


def test_forest_adjoint_matches_single_trees_and_oracle():
    api = _api()
    import torch
    scs = mixed_scenes()
    F = api.Forest(scs)
    acts = _actives(scs, 0.5, seed=70)
    a = F.flat_active(acts)
    rng = np.random.default_rng(3)
    gJ_parts = []
    for sc, act in zip(scs, acts):
        g = rng.normal(size=(sc.n_bands, sc.n))
        g[:, ~act.astype(bool)] = 0.0
        gJ_parts.append(g)
    gJ = torch.as_tensor(np.concatenate([g.ravel() for g in gJ_parts]), device="cuda")
    F.compute_J(a)
    gL, gk, gr = F.compute_J_backward(gJ, a)     # reuses the forward's state
    F.check()
    gLp = [p.cpu().numpy() for p in F.split(gL)]
    gkp = [p.cpu().numpy() for p in F.split(gk)]
    grp = [p.cpu().numpy() for p in F.split(gr)]
    for s, (sc, act) in enumerate(zip(scs, acts)):
        T = F.scene_tree(s)
        bg = None
        if sc.background:
            bg = torch.as_tensor(np.asarray(sc.bg, np.float32), device="cuda")
        aa = torch.as_tensor(act, device="cuda")
        ref = T.compute_J_backward(torch.as_tensor(gJ_parts[s], device="cuda"), aa, bg)
        T.check()
        for got, r in zip((gLp[s], gkp[s], grp[s]), ref):
            _close(got, r.cpu().numpy(), 1e-4)
    # dot product against the oracle's forward-mode derivative, one scene
    s = 1
    sc, act = scs[s], acts[s]
    tk = rng.normal(size=(sc.n_bands, sc.n)) * sc.kappa
    tr = rng.normal(size=sc.n) * sc.rho
    _, dJ, _ = oracle.jvp(sc, tkappa=tk, trho=tr, active=act)
    lhs = float(np.sum(gJ_parts[s] * dJ))
    rhs = float(np.sum(gkp[s] * tk) + np.sum(grp[s] * tr))
    scale = max(float(np.sum(np.abs(gJ_parts[s] * dJ))),
                float(np.sum(np.abs(gkp[s] * tk)) + np.sum(np.abs(grp[s] * tr))))
    assert abs(lhs - rhs) <= 1e-4 * scale, (lhs, rhs, scale)
    F.close()


def test_forest_adjoint_without_forward_state_recomputes_it():
    """A backward on a scratch that holds no forward of this forest redoes
    the forward steps itself; the result equals the reusing one."""
    api = _api()
    import torch
    scs = mixed_scenes()[:4]
    F = api.Forest(scs)
    a = F.flat_active(_actives(scs, 1.0, 0))
    gJ = torch.as_tensor(np.random.default_rng(5).normal(size=int(F.boff[-1])), device="cuda")
    F.compute_J(a)
    r1 = [t.cpu().numpy() for t in F.compute_J_backward(gJ, a)]
    F2 = api.Forest(scs)
    r2 = [t.cpu().numpy() for t in F2.compute_J_backward(gJ, a)]
    F.check()
    F2.check()
    for x, y in zip(r1, r2):
        _close(x, y, 1e-5)
    F.close()
    F2.close()


def test_forest_adjoint_with_a_different_active_set_is_reported():
    api = _api()
    scs = mixed_scenes()[:3]
    F = api.Forest(scs)
    import torch
    a1 = F.flat_active(_actives(scs, 1.0, 0))
    a2 = F.flat_active(_actives(scs, 0.5, 9))
    F.compute_J(a1)
    gJ = torch.zeros(int(F.boff[-1]), dtype=torch.float64, device="cuda")
    outs = F.compute_J_backward(gJ, a2)
    # the gradients of the wrong active set are not left plausible: NaN
    for g in outs:
        assert bool(torch.all(torch.isnan(g)))
    with pytest.raises(api.TrevrError):
        F.check()
    F.close()


def test_forest_profile_records_every_phase():
    """Kernel timing of the batched calls: every phase of a forward and an
    adjoint is timed, one launch per band count for the per-bucket kernels,
    the p-p source kernels inside the near-field totals."""
    api = _api()
    scs = mixed_scenes()[:4]
    F = api.Forest(scs)
    import torch
    a = F.flat_active(_actives(scs, 1.0, 0))
    gJ = torch.as_tensor(np.random.default_rng(3).normal(size=int(F.boff[-1])), device="cuda")
    F.profile(True)
    F.compute_J(a)
    F.compute_J_backward(gJ, a)
    p = F.profile_read()
    F.profile(False)
    F.check()
    nclass = len(set(int(s.n_bands) for s in scs))
    for k in ("setup", "walk", "reduce", "pp_src", "adj_reduce", "adj_pp_src", "adj_tree"):
        assert p[k][1] > 0 and p[k][0] > 0.0, k
    assert p["pp_src"][1] == nclass and p["reduce"][1] == nclass
    assert p["near"][0] >= p["pp_src"][0] and p["adj_near"][0] >= p["adj_pp_src"][0]
    F.close()


def test_forest_graph_of_forward_and_adjoint():
    api = _api()
    import torch
    scs = mixed_scenes()
    F = api.Forest(scs)
    a = F.flat_active(_actives(scs, 1.0, 0))
    gJ = torch.as_tensor(np.random.default_rng(8).normal(size=int(F.boff[-1])), device="cuda")
    J = F.new_J()
    outs = (torch.empty_like(gJ), torch.empty_like(gJ),
            torch.empty(int(F.offsets[-1]), dtype=torch.float64, device="cuda"))
    F.compute_J(a, out=J)
    F.compute_J_backward(gJ, a, out=outs)
    torch.cuda.synchronize()
    ref = [J.cpu().numpy()] + [t.cpu().numpy() for t in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        F.compute_J(a, out=J)
        F.compute_J_backward(gJ, a, out=outs)
    for rep in range(3):
        J.zero_()
        for t in outs:
            t.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = [J.cpu().numpy()] + [t.cpu().numpy() for t in outs]
        F.check()
        assert np.max(_rel(got[0], ref[0])) <= SAME_TOL
        for x, y in zip(got[1:], ref[1:]):
            _close(x, y, 1e-5)
    F.close()


def _log_scenes():
    """Small mixed scenes plus p-p sets of thousands (log-normal, N_side 4)
    and two receiver chunks per bucket (leaf size 12)."""
    return mixed_scenes()[:4] + [
        scenes.lognormal_scene(n=2 ** 13, seed=21, grid=16, bands=(1.0, 10.0), nside=4),
        scenes.lognormal_scene(n=3000, seed=22, grid=16, bands=(1.0,), nside=2, leaf_size=12),
    ]


def test_forest_job_log_gives_the_same_results():
    """With the p-p job log the adjoint runs the forward's own jobs instead
    of culling again: J, gL, gkappa and grho equal those without the log (to
    FP32 rounding of atomic sums) -- with room for every bucket, with room
    for a few (most buckets culled again), on the backward that recomputes
    the forward state, and in a replayed HIP graph of both calls."""
    api = _api()
    import torch
    scs = _log_scenes()
    F = api.Forest(scs)
    acts = _actives(scs, 0.6, seed=31)
    a = F.flat_active(acts)
    gJ = torch.as_tensor(np.random.default_rng(9).normal(size=int(F.boff[-1])), device="cuda")
    J0 = F.compute_J(a).cpu().numpy()
    g0 = [t.cpu().numpy() for t in F.compute_J_backward(gJ, a)]
    F.check()
    c0 = F.counters(-1)
    need = c0["pp_log_entries"]
    assert need > 0

    def same(J, g):
        assert np.max(_rel(J, J0)) <= SAME_TOL
        for x, y in zip(g, g0):
            _close(x, y, 1e-5)

    for nbytes in (2 * need + (64 << 20), 6 * 32768):
        F.set_job_log(nbytes)
        J = F.compute_J(a).cpu().numpy()
        g = [t.cpu().numpy() for t in F.compute_J_backward(gJ, a)]
        F.check()
        same(J, g)
        assert F.counters(-1) == c0
    # a backward with no forward state before it writes and reads the log itself
    F.set_job_log(2 * need + (64 << 20))
    same(J0, [t.cpu().numpy() for t in F.compute_J_backward(gJ, a)])
    F.check()
    # graph of forward and adjoint, replayed with other work between replays
    Jd = F.new_J()
    outs = (torch.empty_like(gJ), torch.empty_like(gJ),
            torch.empty(int(F.offsets[-1]), dtype=torch.float64, device="cuda"))
    F.compute_J(a, out=Jd)
    F.compute_J_backward(gJ, a, out=outs)
    torch.cuda.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        F.compute_J(a, out=Jd)
        F.compute_J_backward(gJ, a, out=outs)
    for rep in range(3):
        Jd.zero_()
        for t in outs:
            t.zero_()
        gr.replay()
        torch.cuda.synchronize()
        F.check()
        same(Jd.cpu().numpy(), [t.cpu().numpy() for t in outs])
        F.compute_J(F.flat_active(_actives(scs, 1.0, 0)))   # eager work between replays
    F.close()


def test_forest_launch_configurations_agree_and_autotune_picks_one():
    """Every launch configuration of the autotuner gives the same J (to FP32
    rounding of atomic sums) and the same gradients; the autotuner times all
    of them and keeps the fastest."""
    api = _api()
    import torch
    scs = mixed_scenes()
    F = api.Forest(scs)
    a = F.flat_active(_actives(scs, 0.5, 21))
    gJ = torch.as_tensor(np.random.default_rng(4).normal(size=int(F.boff[-1])), device="cuda")
    ref = None
    for k in range(api.CONFIGS):
        F.set_config(k)
        J = F.compute_J(a).cpu().numpy()
        g = [t.cpu().numpy() for t in F.compute_J_backward(gJ, a)]
        F.check()
        if ref is None:
            ref = (J, g)
            continue
        assert np.max(_rel(J, ref[0])) <= SAME_TOL, k
        for x, y in zip(g, ref[1]):
            _close(x, y, 1e-5)
    chosen, times = F.autotune(a, gJ=gJ, reps=1)
    F.check()
    assert 0 <= chosen < api.CONFIGS
    assert np.all(times > 0) and times[chosen] == times.min()
    J = F.compute_J(a).cpu().numpy()
    assert np.max(_rel(J, ref[0])) <= SAME_TOL
    F.close()


def test_full_batched_workload_against_the_oracle_sampled():
    """The 64-scene workload, all active, batched on the GPU, against the
    oracle on 96 random receivers of every scene (J of a receiver does not
    depend on which others are active), and, per scene, the batched adjoint
    of weights on those receivers against the oracle's forward-mode
    derivative along random L, kappa and rho directions."""
    api = _api()
    import torch
    scs = scenes.batched_scenes(64)
    F = api.Forest(scs)
    a = F.flat_active([None] * F.S)
    J = F.split(F.compute_J(a))
    F.check()
    rng = np.random.default_rng(123)
    gparts, samples = [], []
    for s, sc in enumerate(scs):
        sub = np.zeros(sc.n, np.uint8)
        sub[rng.choice(sc.n, size=min(96, sc.n), replace=False)] = 1
        samples.append(sub)
        g = rng.normal(size=(sc.n_bands, sc.n))
        g[:, ~sub.astype(bool)] = 0.0
        gparts.append(g)
    gJ = torch.as_tensor(np.concatenate([g.ravel() for g in gparts]), device="cuda")
    gL, gk, gr = (F.split(x) for x in F.compute_J_backward(gJ, a))
    F.check()
    worst = 0.0
    for s, sc in enumerate(scs):
        m = samples[s].astype(bool)
        Jo, _ = oracle.OracleTree(sc).compute_J(samples[s])
        Jg = J[s].cpu().numpy()
        e = float(np.max(_rel(Jg[:, m], Jo[:, m])))
        worst = max(worst, e)
        assert e < J_TOL, (sc.name, e)
        tL = rng.normal(size=(sc.n_bands, sc.n)) * sc.lum
        tk = rng.normal(size=(sc.n_bands, sc.n)) * sc.kappa
        tr = rng.normal(size=sc.n) * sc.rho
        _, dJ, _ = oracle.jvp(sc, tL=tL, tkappa=tk, trho=tr, active=samples[s])
        lhs = float(np.sum(gparts[s] * dJ))
        terms = [gL[s].cpu().numpy() * tL, gk[s].cpu().numpy() * tk, gr[s].cpu().numpy() * tr]
        rhs = float(sum(np.sum(x) for x in terms))
        scale = max(float(np.sum(np.abs(gparts[s] * dJ))),
                    float(sum(np.sum(np.abs(x)) for x in terms)))
        assert abs(lhs - rhs) <= 1e-4 * scale, (sc.name, lhs, rhs, scale)
    print(f"[forest] 64 scenes x 96 receivers: max rel err {worst:.2e}")
    F.close()
