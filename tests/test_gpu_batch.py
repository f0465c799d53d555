"""Batched form on the GPU: many uneven instances advanced by one launch per
step (replayed from a captured graph) give bit-identical states to the same
instances stepped alone, whatever the membership changes in between."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2007_07347_amd import sdugks
    return sdugks


def members(sd):
    """Uneven instances: quads and triangles, FP64 and both FP32 storage forms,
    different viscosities, lids and tile schedules."""
    specs = [
        (meshgen.cavity(23), dict(nu=1e-3)),
        (meshgen.cavity(40, U=0.05), dict(nu=4e-4, tile_cells=16, block_threads=64)),
        (meshgen.cavity(64), dict(nu=2e-4, precision=sd.FP32DEV)),
        (meshgen.cylinder_ogrid(48, 16, seed=3), dict(nu=2.5e-3, u0=0.1)),
        (meshgen.jittered_periodic_triangles(12, seed=4), dict(nu=4e-3, precision=sd.FP32DEV)),
        (meshgen.couette(4, 32), dict(nu=1e-2, macro=sd.MACRO_LAGGED, cfl=0.3)),
        (meshgen.cylinder_ogrid(40, 12, seed=7, quad_layers=4), dict(nu=2.5e-3, u0=0.1, precision=sd.FP32DEV)),
        (meshgen.cavity(31), dict(nu=5e-4, precision=sd.FP32NEQ)),
        (meshgen.cylinder_ogrid(36, 10, seed=9), dict(nu=2.5e-3, u0=0.1, precision=sd.FP32NEQ)),
    ]
    return specs


def make(sd, specs, seed):
    out = []
    for k, ((mesh, bcs), kw) in enumerate(specs):
        s = sd.Solver(mesh, bcs, cfl=kw.pop("cfl", 0.5), **kw)
        f, W, _ = meshgen.random_state(s.n_cells, seed=seed + k, amp=0.01)
        s.set_state(f, W)
        out.append(s)
    return out


def states(solvers):
    return [s.state() for s in solvers]


def assert_same(a, b):
    for sa, sb in zip(a, b):
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y)


# step counts that replay every graph length: 30 = 8 + 4 + 2 + 1 pairs, 95 =
# two 16-pair runs + 8 + 4 + 2 + 1 pairs + an odd step
@pytest.mark.parametrize("n", [1, 2, 7, 30, 40, 95])
def test_batch_equals_alone(sd, n):
    alone = make(sd, members(sd), seed=100)
    batched = make(sd, members(sd), seed=100)
    for s in alone:
        s.step(n)
    b = sd.Batch(batched)
    b.step(n)
    assert_same(states(alone), states(batched))
    b.close()


def test_graph_replays_with_eager_work_between(sd):
    """Graph replays interleaved with members stepped alone, residual and mass
    reductions and host synchronisations: every replay matches the eager run."""
    alone = make(sd, members(sd), seed=200)
    batched = make(sd, members(sd), seed=200)
    b = sd.Batch(batched)
    for rnd in range(5):
        for s in alone:
            s.step(6)
        b.step(6)
        assert_same(states(alone), states(batched))
        # eager work on one member between replays
        alone[1].step(3)
        batched[1].step(3)
        alone[1].residual()
        batched[1].residual()
        assert batched[2].mass() == alone[2].mass()
    b.close()


@pytest.mark.parametrize("steps", [5, 37])
def test_continuous_batching_membership_changes(sd, steps):
    """Members join and leave between steps (admission / retirement; members
    that need more LDS than the launch was captured with force a rebuild):
    results stay bitwise those of stepping each instance alone, both with
    short runs and with runs long enough to replay the long graph."""
    specs = members(sd)
    alone = make(sd, specs, seed=300)
    batched = make(sd, members(sd), seed=300)
    b = sd.Batch(batched[:2])
    plan = [[0, 1], [0, 1, 2, 3], [1, 3, 4], [0, 1, 2, 3, 4, 5], [5], [2, 4]]
    for ids in plan:
        b.set_members([batched[k] for k in ids])
        b.step(steps)
        for k in ids:
            alone[k].step(steps)
    assert_same(states(alone), states(batched))
    b.close()


def test_batch_rejects_two_kernel_members(sd):
    hexes = sd.Solver(*meshgen.hexagon_strip(4, 3), nu=0.01)
    cav = sd.Solver(*meshgen.cavity(8), nu=0.01)
    with pytest.raises(sd.SdugksError):
        sd.Batch([cav, hexes])
    with pytest.raises(sd.SdugksError):
        sd.Batch([cav, cav])


def test_batch_refuses_diverged_member(sd):
    a = sd.Solver(*meshgen.cavity(12), nu=2e-3)
    c = sd.Solver(*meshgen.cavity(10), nu=2e-3)
    b = sd.Batch([a, c])
    b.step(4)
    a.poison(5, 2)
    a.step(1)
    with pytest.raises(sd.SdugksError):
        a.residual()
    with pytest.raises(sd.SdugksError) as ei:
        b.step(2)
    assert ei.value.code == sd.EDIVERGED
    b.set_members([c])
    b.step(2)
    c.residual()
    b.close()


def test_batch_autotuner_times_every_candidate(sd, tmp_path):
    """The batch autotuner applies each candidate schedule to every member,
    times the batched step, returns the fastest and caches the choice."""
    from paper_2007_07347_amd import autotune
    problems = [(*meshgen.cavity(n), dict(nu=1e-3, cfl=0.5, precision=sd.FP32DEV)) for n in (24, 40, 57)]
    cands = [(32, 128), (64, 256)]
    cache = str(tmp_path / "cache.json")
    best, table = autotune.autotune_batch(problems, candidates=cands, steps=5, cache=cache)
    assert [(r["tile_cells"], r["block_threads"]) for r in table] == cands
    assert all(r["ms"] is not None and r["ms"] > 0 for r in table)
    fastest = min(table, key=lambda r: r["ms"])
    assert best == {"tile_cells": fastest["tile_cells"], "block_threads": fastest["block_threads"], "structured": 1}
    again, _ = autotune.autotune_batch(problems, candidates=cands, steps=5, cache=cache)
    assert again == best
    # without a candidate list, tensor-product meshes also try the structured step
    best, table = autotune.autotune_batch(problems, steps=5, cache=None)
    assert table[0]["structured"] == 2 and len(table) == 1 + len(autotune.CANDIDATES)
    assert autotune.label(best) in {autotune.label(r) for r in table}


@pytest.mark.parametrize("sched", ["structured", (64, 256), (32, 128)])
def test_full_size_64_cavity_batch(sd, oracle_mod, sched):
    """The batched workload at its full size (64 tanh cavities, edges
    log-uniform in [32, 512], Re uniform in [100, 5000], seed 2026, FP32
    deviation storage, 2.29M cells) on the schedules the batch autotuner
    chooses between (the structured step, which it picks, and the general
    step's best two): 30 batched steps give the same bits as each member
    stepped alone, and the two smallest members, sampled against the FP64
    oracle, stay within the FP32 deviation form's window bar."""
    rng = np.random.default_rng(2026)
    sizes = meshgen.log_uniform_int(rng, 32, 512, size=64)
    res = rng.uniform(100.0, 5000.0, size=64)
    sk = dict(structured=2) if sched == "structured" else dict(tile_cells=sched[0], block_threads=sched[1])
    problems = [(meshgen.cavity(int(n), beta=1.5, U=0.1), dict(nu=0.1 / re, cfl=0.5)) for n, re in zip(sizes, res)]
    assert sum(int(n) ** 2 for n in sizes) == 2289523
    mk = lambda: [sd.Solver(m, b, precision=sd.FP32DEV, **sk, **kw)
                  for (m, b), kw in problems]
    alone, batched = mk(), mk()
    for s in alone:
        s.step(30)
    b = sd.Batch(batched)
    b.step(30)
    for k in range(64):
        for x, y in zip(alone[k].state(), batched[k].state()):
            assert np.array_equal(x, y), k
    b.close()
    for k in np.argsort(sizes, kind="stable")[:2]:
        (m, bc), kw = problems[k]
        o = oracle_mod.Oracle(m, bc, **kw)
        o.step(30)
        fg, Wg, _ = batched[k].state()
        fo, Wo, _ = o.state()
        ef = np.abs(fg - fo).max() / np.abs(fo).max()
        ew = np.abs(Wg - Wo).max() / np.abs(Wo).max()
        assert ef <= 2e-6 and ew <= 2e-6, (k, ef, ew)
    for s in alone + batched:
        s.close()


def test_members_on_their_own_streams(sd):
    """Members enqueue on streams of their own and the batch on another: the
    batch waits for work each member queued before it, and each member's
    later work waits for the batch, so the interleaving gives the same bits
    as stepping every instance alone on one stream."""
    import torch
    specs = members(sd)[:4]
    alone = make(sd, members(sd)[:4], seed=400)
    streams = [torch.cuda.Stream() for _ in specs]
    batched = []
    for k, ((mesh, bcs), kw) in enumerate(specs):
        kw = dict(kw)
        s = sd.Solver(mesh, bcs, stream=streams[k], cfl=kw.pop("cfl", 0.5), **kw)
        f, W, _ = meshgen.random_state(s.n_cells, seed=400 + k, amp=0.01)
        s.set_state(f, W)
        batched.append(s)
    b = sd.Batch(batched, stream=torch.cuda.Stream())
    for rnd in range(4):
        for k, s in enumerate(batched):       # queued, not waited for
            s.step(k + 1)
        b.step(5 + rnd)
        for s in batched[::2]:
            s.step(2)
        for k, s in enumerate(alone):
            s.step(k + 1)
            s.step(5 + rnd)
        for s in alone[::2]:
            s.step(2)
    assert_same(states(alone), states(batched))
    b.close()
