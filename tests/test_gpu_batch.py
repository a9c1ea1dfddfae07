"""Batched solves through ``ddg_setup_batched`` / ``ddg_solve_batched``.

Every system of a batch must behave as if it were solved alone: the
preconditioner applied to the concatenated residual equals, system by
system, the FP64 oracle's M^{-1} of that system (1e-12 relative); the batched
FP64 solve matches the oracle's PCG per system (u within 1e-10 relative,
iterations +-1) and a standalone handle of the same system (same iteration
count); mixed FP32 reaches true residual <= 1e-8 per system.  Systems
stop independently: a zero right-hand side stops at iteration 0 and an
iteration cap stops only the systems that need more.
"""

import sys

import numpy as np
import pytest

from oracle import DDGOracle
from parity_util import FP64_U_TOL, fp64_u_error
from workloads import cfg4_instance, seed_rng

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# uneven sizes: 1x1 .. 4x4 boxes of about 16 cells, overlap 2, p = 3 (the batched workload's
# settings at a size the oracle finishes quickly)
SIDES = [12, 21, 30, 37, 46, 64]
_cache = {}


def systems():
    if "s" not in _cache:
        Ps = [cfg4_instance(100 + i, L, overlap=2, p=3, cell=16, rtol=1e-10) for i, L in enumerate(SIDES)]
        Os = [DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap) for P in Ps]
        _cache["s"] = (Ps, Os)
    return _cache["s"]


def make_batch(Ps, **kw):
    from paper_1504_00907_amd import DDGBatchSolver
    say(f"[batch setup] {len(Ps)} systems, n = {[P.n for P in Ps]} {kw}")
    probs = [(P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts) for P in Ps]
    return DDGBatchSolver(probs, Ps[0].overlap, **kw)


def test_layout_and_structures():
    Ps, Os = systems()
    b = make_batch(Ps)
    assert b.nb == len(Ps)
    assert list(np.diff(b.row_off)) == [P.n for P in Ps]
    assert list(np.diff(b.sub_off)) == [P.n_parts for P in Ps]
    kc = b.kcounts()
    for i, (P, o) in enumerate(zip(Ps, Os)):
        assert np.array_equal(kc[b.sub_off[i]:b.sub_off[i + 1]], o.k_counts)
    # colours of each system's subdomains equal its own greedy colouring
    col = b.colours()
    for i, o in enumerate(Os):
        assert np.array_equal(col[b.sub_off[i]:b.sub_off[i + 1]], o.colours)
    # A0 blocks: one per system, spectrum equal to the oracle's
    a0 = b.export(4)
    off = 0
    for P, o in zip(Ps, Os):
        m = o.n_coarse
        A0 = a0[off:off + m * m].reshape(m, m)
        off += m * m
        ev = np.sort(np.linalg.eigvalsh(0.5 * (A0 + A0.T)))
        ev_ref = np.sort(np.linalg.eigvalsh(o.A0))
        assert np.abs(ev - ev_ref).max() <= 1e-11 * ev_ref.max()
    assert off == a0.size
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_preconditioner_per_system(precision):
    Ps, Os = systems()
    b = make_batch(Ps, precision=precision)
    rng = seed_rng(80, 0)
    rs = [rng.standard_normal(P.n) for P in Ps]
    z = host(b.apply_precond(dev(np.concatenate(rs))))
    tol = 1e-12 if precision == "fp64" else 1e-5
    for i, (o, r) in enumerate(zip(Os, rs)):
        zi = z[b.row_off[i]:b.row_off[i + 1]]
        ref = o.apply(r)
        err = np.linalg.norm(zi - ref) / np.linalg.norm(ref)
        say(f"   system {i} (n={r.size}) rel err {err:.2e}")
        assert err <= tol
    b.close()


def test_fp64_solve_matches_oracle_and_standalone():
    from paper_1504_00907_amd import DDGSolver
    Ps, Os = systems()
    b = make_batch(Ps, rtol=1e-10)
    f = np.concatenate([P.f for P in Ps])
    u, infos = b.solve(dev(f))
    u = host(u)
    for i, (P, o) in enumerate(zip(Ps, Os)):
        ui = u[b.row_off[i]:b.row_off[i + 1]]
        x, it, _ = o.pcg(P.f, 1e-10)
        err = np.linalg.norm(ui - x) / np.linalg.norm(x)
        s = DDGSolver.from_problem(P, rtol=1e-10)
        us, info_s = s.solve(dev(P.f))
        s.close()
        say(f"   system {i}: iters batch {infos[i]['iters']} alone {info_s['iters']} oracle {it}, "
            f"err {err:.2e}, solve_ms {infos[i]['solve_ms']:.2f}")
        assert infos[i]["status"] == 0
        assert infos[i]["iters"] == info_s["iters"]

        def rerun(m, P=P):
            s2 = DDGSolver.from_problem(P, rtol=0.0, max_iter=m)
            um, im = s2.solve(dev(P.f), raise_on_error=False)
            assert im["iters"] == m
            um = host(um)
            s2.close()
            return um

        err, at = fp64_u_error(ui, infos[i]["iters"], x, it, rerun, lambda m, o=o, P=P: o.pcg(P.f, 0.0, m)[0])
        assert err <= FP64_U_TOL
        assert np.linalg.norm(ui - host(us)) <= 1e-12 * np.linalg.norm(ui)
        true_res = np.linalg.norm(P.f - P.A.to_scipy() @ ui) / np.linalg.norm(P.f)
        assert abs(true_res - infos[i]["true_rel_res"]) <= 1e-3 * true_res + 1e-15
        assert infos[i]["n_coarse"] == o.n_coarse and infos[i]["n_parts"] == P.n_parts
        assert 0.0 < infos[i]["solve_ms"]
    b.close()


def test_mixed_solve_per_system():
    Ps, Os = systems()
    b = make_batch(Ps, rtol=1e-8, precision="fp32")
    f = np.concatenate([P.f for P in Ps])
    u, infos = b.solve(dev(f))
    u = host(u)
    for i, (P, o) in enumerate(zip(Ps, Os)):
        ui = u[b.row_off[i]:b.row_off[i + 1]]
        true_res = np.linalg.norm(P.f - P.A.to_scipy() @ ui) / np.linalg.norm(P.f)
        _, it, _ = o.pcg(P.f, 1e-8)
        say(f"   system {i}: iters {infos[i]['iters']} (oracle fp64 {it}) true res {true_res:.2e}")
        assert infos[i]["status"] == 0 and true_res <= 1e-8
        assert abs(infos[i]["iters"] - it) <= 1
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_task_queue_schedule_matches_colour_launches(precision):
    """The task-queue schedule over the whole batch (tasks of all systems in one
    queue, converged systems skipped) gives the colour-by-colour results bit for bit."""
    Ps, Os = systems()
    f = dev(np.concatenate([P.f for P in Ps]))
    out = []
    for schedule in ("queue", "colours"):
        b = make_batch(Ps, precision=precision, rtol=1e-8, schedule=schedule)
        u, infos = b.solve(f)
        out.append((host(u), [i["iters"] for i in infos]))
        b.close()
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def test_systems_stop_independently():
    from paper_1504_00907_amd import DDGError
    Ps, Os = systems()
    b = make_batch(Ps, rtol=1e-10)
    fs = [P.f.copy() for P in Ps]
    fs[2][:] = 0.0
    u, infos = b.solve(dev(np.concatenate(fs)))
    u = host(u)
    assert infos[2]["iters"] == 0 and infos[2]["status"] == 0
    assert not np.any(u[b.row_off[2]:b.row_off[3]])
    assert all(infos[i]["iters"] > 0 for i in range(len(Ps)) if i != 2)
    b.close()
    # an iteration cap below the largest system's count stops only the systems that need more
    b = make_batch(Ps, rtol=1e-10)
    _, full = b.solve(dev(np.concatenate([P.f for P in Ps])))
    cap = sorted(i["iters"] for i in full)[len(Ps) // 2]
    b.close()
    b = make_batch(Ps, rtol=1e-10, max_iter=cap)
    u, infos = b.solve(dev(np.concatenate([P.f for P in Ps])), raise_on_error=False)
    for i, P in enumerate(Ps):
        if full[i]["iters"] <= cap:
            assert infos[i]["status"] == 0 and infos[i]["iters"] == full[i]["iters"]
        else:
            assert infos[i]["status"] == -5 and infos[i]["iters"] == cap
    with pytest.raises(DDGError):
        b.solve(dev(np.concatenate([P.f for P in Ps])))
    b.close()


def test_autotuner_picks_a_measured_shape(tmp_path):
    from paper_1504_00907_amd import DDGBatchSolver, tune_batched
    Ps, Os = systems()
    probs = [(P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts) for P in Ps]
    cache = str(tmp_path / "tune.txt")
    tile, bt, cands = tune_batched(probs, 2, "fp32", max_sample=4, cache=cache)
    say(f"   tuner: tile {tile} block_target {bt}; candidates {cands}")
    assert len(cands) == 9
    timed = [c for c in cands if c[2] >= 0]
    assert timed and min(timed, key=lambda c: c[2])[:2] == (tile, bt)
    # a cache hit returns the same choice without measuring
    tile2, bt2, cands2 = tune_batched(probs, 2, "fp32", max_sample=4, cache=cache)
    assert (tile2, bt2) == (tile, bt) and cands2 == []
    # the chosen shape solves the batch like the default one
    b = DDGBatchSolver(probs, 2, precision="fp32", rtol=1e-8, tile=tile, block_target=bt)
    u, infos = b.solve(dev(np.concatenate([P.f for P in Ps])))
    u = host(u)
    for i, P in enumerate(Ps):
        ui = u[b.row_off[i]:b.row_off[i + 1]]
        assert np.linalg.norm(P.f - P.A.to_scipy() @ ui) <= 1e-8 * np.linalg.norm(P.f)
    b.close()


@pytest.mark.slow
def test_full_batch_sampled():
    """The 256-system batch of the benchmark (FP32 factors, rtol 1e-8): every system
    reaches the residual; sampled systems (smallest, largest, two seeded) match a
    standalone handle's iteration count and the FP64 oracle's (+-1)."""
    import multiprocessing as mp
    from paper_1504_00907_amd import DDGBatchSolver, DDGSolver
    from workloads import cfg4_sides
    sides = cfg4_sides()
    with mp.get_context("spawn").Pool(16) as pool:
        Ps = pool.starmap(cfg4_instance, [(i, int(L)) for i, L in enumerate(sides)], chunksize=4)
    probs = [(P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts) for P in Ps]
    say(f"[batch] {len(Ps)} systems, n = {sum(P.n for P in Ps)}")
    b = DDGBatchSolver(probs, 2, precision="fp32", rtol=1e-8)
    u, infos = b.solve(dev(np.concatenate([P.f for P in Ps])))
    u = host(u)
    assert all(i["status"] == 0 for i in infos)
    assert max(i["true_rel_res"] for i in infos) <= 1e-8
    b.close()
    order = np.argsort(sides)
    rng = seed_rng(81, 0)
    picks = [int(order[0]), int(order[-1])] + [int(x) for x in rng.choice(len(Ps), 2, replace=False)]
    for i in picks:
        P = Ps[i]
        ui = u[b.row_off[i]:b.row_off[i + 1]]
        true_res = np.linalg.norm(P.f - P.A.to_scipy() @ ui) / np.linalg.norm(P.f)
        s = DDGSolver.from_problem(P, precision="fp32", rtol=1e-8)
        us, info_s = s.solve(dev(P.f))
        s.close()
        o = DDGOracle(P.A, P.F, P.part, P.n_parts, P.overlap)
        x, it, _ = o.pcg(P.f, 1e-8)
        say(f"   system {i} (L={sides[i]}, n={P.n}): iters batch {infos[i]['iters']} alone {info_s['iters']} "
            f"oracle {it}, true res {true_res:.2e}")
        assert true_res <= 1e-8
        assert infos[i]["iters"] == info_s["iters"] and abs(infos[i]["iters"] - it) <= 1
        assert np.linalg.norm(ui - host(us)) <= 1e-8 * np.linalg.norm(ui)
