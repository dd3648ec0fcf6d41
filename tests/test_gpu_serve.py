"""The request loop on the GPU: requests for two resident ensembles of
different volumes arrive while others run, join the running multi-rhs solves
between outer cycles (continuous batching through the library's slot pool,
requests larger than the free slots in parts), and each result equals the
same request computed alone."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ENS = {
    "8^4": dict(L=(8, 8, 8, 8), block=(4, 4, 4, 4), eps=0.3, kappa=0.124, csw=1.0, Nv=6, Nlm=2, seed=11),
    "16x8^3": dict(L=(16, 8, 8, 8), block=(4, 4, 4, 4), eps=0.3, kappa=0.124, csw=1.0, Nv=6, Nlm=2, seed=12),
}


def test_serving_alone_equals_mix():
    import torch
    from paper_2412_06347_amd.serve import Server, Engine, poisson_arrivals
    free, _ = torch.cuda.mem_get_info()
    srv = Server(hbm_budget=0.5 * free, max_batch_rhs=16)
    for name, wl in ENS.items():
        srv.add_ensemble(name, wl)
    srv.start()
    # arrivals a few milliseconds apart, well inside one batch's service time,
    # so requests arrive while others are on the GPU
    arr = poisson_arrivals(12, 400.0, 5)
    reqs = []
    t0 = time.perf_counter()
    for i, t in enumerate(arr):
        while time.perf_counter() - t0 < t:
            time.sleep(0.001)
        reqs.append(srv.submit(list(ENS)[i % 2], 1 + i % 3, 100 + i))
    for r in reqs:
        r.wait(300)
    srv.stop()
    st = srv.stats()
    print("serving stats", st, "batches", srv.batches)
    assert st["n"] == len(reqs) and st["p99_s"] >= st["p50_s"] > 0
    assert any(len(b) > 1 for b in srv.batches)          # requests shared outer cycles
    # a request admitted while another was running started before that one ended
    joined = [(r, q) for r in reqs for q in reqs
              if r.ensemble == q.ensemble and q.t_start < r.t_start < q.t_done and r.joined_running > 0]
    print("requests that joined a running solve:", len(joined))
    assert joined
    # each result equals the same request run alone
    for r in reqs:
        eng = srv.engines[r.ensemble]
        alone = eng.run([r])[0]
        for key in ("L0", "L1", "L2"):
            a, b = alone[key], r.result[key]
            assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a)), (r.rid, key)
        assert r.result["max_true_rel_res"] <= 1e-10
