"""Persistent batched solve (schedule "persistent": the whole PCG of every system
in one launch, systems advancing through their own steps from a device task ring).

With one workgroup per subdomain (DDG_NO_TWIST), the persistent launch gives the
colour-launch results bit for bit: u, iteration counts, statuses and the CG
histories, in every precision mode and both direction updates.  With the default
two-workgroup colour launches the solutions agree to 1e-12 at equal iteration
counts.  Systems stop independently (zero right-hand side, iteration cap), and
their solve times differ: a small system finishes before a large one.
"""

import sys

import numpy as np
import pytest

from workloads import cfg1, cfg4_instance, diffusion_problem

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# uneven sizes and subdomain counts: the systems need different iteration counts and
# finish at different times
SIDES = [12, 21, 30, 37, 46, 64]
_cache = {}


def systems():
    if "s" not in _cache:
        _cache["s"] = [cfg4_instance(200 + i, L, overlap=2, p=3, cell=16, rtol=1e-10) for i, L in enumerate(SIDES)]
    return _cache["s"]


def batch(Ps, **kw):
    from paper_1504_00907_amd import DDGBatchSolver
    say(f"[batch setup] {len(Ps)} systems, n = {[P.n for P in Ps]} {kw}")
    probs = [(P.A.row_ptr, P.A.col_idx, P.A.val, P.F, P.part, P.n_parts) for P in Ps]
    return DDGBatchSolver(probs, Ps[0].overlap, **kw)


def run(b, f, raise_on_error=True):
    u, infos = b.solve(f, raise_on_error=raise_on_error)
    hist = [b.cg_history(i) for i in range(b.nb)]
    return host(u), infos, hist


@pytest.mark.parametrize("precision,variant", [("fp64", "fr"), ("fp32", "fr"), ("bf16", "fr"), ("fp32", "pr")])
def test_persistent_matches_colour_launches_bitwise(precision, variant, monkeypatch):
    monkeypatch.setenv("DDG_NO_TWIST", "1")
    Ps = systems()
    f = dev(np.concatenate([P.f for P in Ps]))
    out = {}
    for schedule in ("persistent", "colours"):
        b = batch(Ps, precision=precision, rtol=1e-10, schedule=schedule, cg_variant=variant)
        assert b.info()["schedule"] == (3 if schedule == "persistent" else 1)
        out[schedule] = run(b, f)
        b.close()
    up, ip, hp = out["persistent"]
    uc, ic, hc = out["colours"]
    say(f"   iters persistent {[i['iters'] for i in ip]} colours {[i['iters'] for i in ic]}")
    assert [i["iters"] for i in ip] == [i["iters"] for i in ic]
    assert [i["status"] for i in ip] == [i["status"] for i in ic] == [0] * len(Ps)
    assert np.array_equal(up, uc)
    for a, c in zip(hp, hc):
        for x, y in zip(a, c):
            assert np.array_equal(x, y)
    assert [i["true_rel_res"] for i in ip] == [i["true_rel_res"] for i in ic]


def test_persistent_matches_two_workgroup_colour_launches():
    Ps = systems()
    f = dev(np.concatenate([P.f for P in Ps]))
    res = {}
    for schedule in ("persistent", "colours"):
        b = batch(Ps, precision="fp64", rtol=1e-10, schedule=schedule)
        u, infos, _ = run(b, f)
        res[schedule] = (u, [i["iters"] for i in infos])
        b.close()
    (up, ip), (uc, ic) = res["persistent"], res["colours"]
    err = np.linalg.norm(up - uc) / np.linalg.norm(uc)
    say(f"   iters {ip} vs {ic}; rel diff {err:.1e} (bitwise equal: {np.array_equal(up, uc)})")
    assert ip == ic and err <= 1e-12


def test_persistent_systems_stop_and_finish_independently(monkeypatch):
    from paper_1504_00907_amd import DDGError
    monkeypatch.setenv("DDG_NO_TWIST", "1")
    Ps = systems()
    # a zero right-hand side stops its system at iteration 0; the others run on
    b = batch(Ps, rtol=1e-10, schedule="persistent")
    fs = [P.f.copy() for P in Ps]
    fs[2][:] = 0.0
    u, infos, _ = run(b, dev(np.concatenate(fs)))
    assert infos[2]["iters"] == 0 and infos[2]["status"] == 0
    assert not np.any(u[b.row_off[2]:b.row_off[3]])
    assert all(infos[i]["iters"] > 0 for i in range(len(Ps)) if i != 2)
    # solve times per system: the smallest system finishes well before the largest
    _, full, _ = run(b, dev(np.concatenate([P.f for P in Ps])))
    ms = [i["solve_ms"] for i in full]
    say(f"   per-system solve ms {[round(x, 3) for x in ms]}, iters {[i['iters'] for i in full]}")
    assert ms[0] < ms[-1]
    b.close()
    # an iteration cap below the largest count stops only the systems that need more
    cap = max(i["iters"] for i in full) - 1
    b = batch(Ps, rtol=1e-10, max_iter=cap, schedule="persistent")
    _, infos, _ = run(b, dev(np.concatenate([P.f for P in Ps])), raise_on_error=False)
    for i in range(len(Ps)):
        if full[i]["iters"] <= cap:
            assert infos[i]["status"] == 0 and infos[i]["iters"] == full[i]["iters"]
        else:
            assert infos[i]["status"] == -5 and infos[i]["iters"] == cap
    with pytest.raises(DDGError):
        b.solve(dev(np.concatenate([P.f for P in Ps])))
    b.close()


@pytest.mark.parametrize("case", ["cfg1", "diffusion3d_k0", "diffusion3d_48"])
def test_persistent_single_system(case, monkeypatch):
    """One system: the 2D Poisson workload, a 3D diffusion problem without a coarse
    space (one-level Schwarz) and a 3D diffusion problem at 48^3 with 64 subdomains."""
    from paper_1504_00907_amd import DDGSolver
    monkeypatch.setenv("DDG_NO_TWIST", "1")
    if case == "cfg1":
        P = cfg1()
    elif case == "diffusion3d_k0":
        P = diffusion_problem((24, 24, 24), (3, 3, 3), 1, 0, cfg_id=7, rtol=1e-8)
        P.F = P.F[:, :0]
    else:
        P = diffusion_problem((48, 48, 48), (4, 4, 4), 1, 2, cfg_id=8, rtol=1e-8)
    out = {}
    for schedule in ("persistent", "colours"):
        s = DDGSolver.from_problem(P, precision="fp32", rtol=P.rtol, schedule=schedule)
        u, inf = s.solve(dev(P.f))
        out[schedule] = (host(u), inf["iters"], inf["status"])
        s.close()
    say(f"   {case}: iters {out['persistent'][1]} vs {out['colours'][1]}")
    assert out["persistent"][1:] == out["colours"][1:]
    assert np.array_equal(out["persistent"][0], out["colours"][0])


def test_persistent_unsupported_configurations():
    from paper_1504_00907_amd import DDGError, DDGSolver
    P = cfg1()
    with pytest.raises(DDGError) as e:
        DDGSolver.from_problem(P, schedule="persistent", local_solver="ssor")
    assert e.value.code == -8


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_persistent_elasticity_matches_colour_launches(precision, monkeypatch):
    """Q1 elasticity (about 78 entries per row): sliced level couplings and lane-group
    row dots inside the persistent kernel; bit for bit the colour launches' results."""
    from paper_1504_00907_amd import DDGSolver
    from workloads.elasticity import elasticity_q1
    monkeypatch.setenv("DDG_NO_TWIST", "1")
    P = elasticity_q1(nel=10, part_dofs=(200, 500), min_dofs=200, sigma=1.0, rtol=1e-10)
    out = {}
    for schedule in ("persistent", "colours"):
        s = DDGSolver.from_problem(P, precision=precision, rtol=P.rtol, schedule=schedule)
        u, inf = s.solve(dev(P.f))
        out[schedule] = (host(u), inf["iters"], inf["status"])
        s.close()
    say(f"   elasticity {precision}: iters {out['persistent'][1]} vs {out['colours'][1]}")
    assert out["persistent"][1:] == out["colours"][1:]
    assert np.array_equal(out["persistent"][0], out["colours"][0])
