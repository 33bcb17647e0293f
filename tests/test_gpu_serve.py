"""Serving loop (needs a GPU): continuous batching of GMRES solves.

Each result served in the mix must equal (bit for bit) the same request
solved alone; admission must respect the device-memory budget; requests
must overlap on the device; an oversized request is refused, not hung.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
U = pytest.importorskip("paper_2501_04684_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    U.lib()
    global S
    import paper_2501_04684_amd.serve as S


def _requests(count=6, lo=150, hi=1500, max_nrhs=3, rate=400.0, seed=7):
    reqs = []
    for i, d in enumerate(W.serving_requests(count, rate, seed, lo, hi, max_nrhs)):
        b = W.complex_normal((d["nrhs"], len(d["boxes"]) * 81), d["b_seed"])
        reqs.append(S.Request(i, d["boxes"], b, arrival=d["arrival"], restart=20,
                              tol=1e-4, max_steps=200))
    return reqs


def _alone(req):
    ff = U.FarField(req.boxes, req.a, req.k, req.n_d, req.far_mode, max_nrhs=req.nrhs,
                    precision=req.precision)
    solver = U.Solver(ff, 0.0, nrhs=req.nrhs, restart=req.restart, tol=req.tol,
                      max_steps=req.max_steps)
    sigma = S.auto_shift(solver)
    x, st = solver.solve(torch.from_numpy(req.b).cuda())
    torch.cuda.synchronize()
    out = x.cpu().numpy(), st, sigma
    solver.close()
    ff.close()
    return out


def test_results_in_the_mix_equal_results_alone():
    reqs = _requests()
    announce("serve mix", [len(r.boxes) for r in reqs], [r.nrhs for r in reqs])
    srv = S.Server(hbm_budget=64 << 30, max_active=8, steps_per_tick=2)
    res = srv.run(reqs, realtime=True)
    srv.close()
    assert srv.peak_active >= 2            # the requests overlapped
    for r, out in zip(reqs, res):
        assert out.error is None and out.converged, (r.rid, out.error)
        x, st, sigma = _alone(r)
        assert sigma == out.sigma
        assert np.array_equal(x, out.x), r.rid
        assert out.max_rel_res <= r.tol
        assert out.t_arrival <= out.t_admit <= out.t_done


def test_admission_respects_budget_and_refuses_oversized():
    reqs = _requests(count=5, seed=8)
    fps = []
    for r in reqs:
        p = U.plan_create(r.boxes, r.a, r.k, r.n_d, r.far_mode, 0.0, r.precision)
        fps.append(S.footprint_bytes(p, r.nrhs, r.restart))
        U.plan_destroy(p)
    budget = int(sorted(fps)[-1] + sorted(fps)[-2])   # two largest fit together
    big = reqs[-1]
    huge = S.Request(99, W.grid_boxes(12, 12, 12), W.complex_normal((8, 12 ** 3 * 81), 3),
                     restart=20)
    announce("serve budget", budget, fps)
    srv = S.Server(hbm_budget=budget, max_active=8)
    res = srv.run(reqs + [huge], realtime=False)
    srv.close()
    by = {o.rid: o for o in res}
    assert by[99].error and "budget" in by[99].error and by[99].x is None
    for r in reqs:
        assert by[r.rid].converged and by[r.rid].error is None
    assert max(in_use for _, _, in_use in srv.log) <= budget
    # the mix under the tight budget still gives the results computed alone
    x, _, _ = _alone(big)
    assert np.array_equal(x, by[big.rid].x)


def test_norm_estimate_against_dense_norm():
    boxes = W.mask_boxes(300, 0.6, 3)
    announce("norm estimate", len(boxes))
    ff = U.FarField(boxes, 0.25, 2 * np.pi, 2)
    s = U.Solver(ff, 0.0, nrhs=1, restart=4)
    est = s.norm_estimate(iters=6, seed=1)
    from oracle import gmres as G
    true = np.linalg.norm(G.far_matrix(boxes, 0.25, 2 * np.pi, 2), 2)
    print("estimate", est, "2-norm", true)
    assert 0.9 * true <= est <= true * (1 + 1e-5)
    assert s.norm_estimate(iters=6, seed=1) == est      # reproducible


def test_served_solution_true_residual():
    r = _requests(count=1, lo=200, hi=300, max_nrhs=1, seed=9)[0]
    announce("serve true residual", len(r.boxes))
    srv = S.Server(hbm_budget=8 << 30, max_active=2)
    out = srv.run([r], realtime=False)[0]
    srv.close()
    x64 = out.x.astype(np.complex128)
    Ax = out.sigma * x64 + O.far_mvm(x64, r.boxes, r.a, r.k, r.n_d)
    b = r.b.astype(np.complex128)
    rel = np.linalg.norm(b - Ax) / np.linalg.norm(b)
    print("true residual", rel, "steps", out.steps)
    assert rel <= 2 * r.tol
