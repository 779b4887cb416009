"""Serving on the GPU: requests of mixed geometries, operations and batch
sizes go through the continuous-batching server (FP32, several streams,
spectra cache) and each result must equal the same request computed alone.

Tolerance: the kernels do not depend on the batch a model is computed in
(the layer split is fixed per geometry), so the results are compared for
exact equality; a served forward is also checked against the oracle at a few
stations to the FP32 bound (1e-5 relative)."""

import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_10160_amd as gf
    return gf


def test_served_equals_alone(gf, orc):
    from paper_2005_10160_amd.serve import GeometryKey, GpuExecutor, Request, Server
    rng = np.random.default_rng(8)
    specs = []
    for i in range(14):
        n = int(rng.choice([64, 128]))
        nz = int(rng.choice([8, 16]))
        comps = 0x3F if rng.random() < 0.5 else 0x1
        op = "forward" if rng.random() < 0.5 else "adjoint"
        B = int(rng.integers(1, 5))
        key = GeometryKey(n, n, nz, 20.0, 20.0, 20.0, 10.0, comps)
        C = key.n_out
        shape = (B, nz, n, n) if op == "forward" else (B, C, n, n)
        x = torch.from_numpy(rng.uniform(-500, 500, size=shape).astype(np.float32)).pin_memory()
        specs.append((key, op, x))
    ex = GpuExecutor("f32", 4)
    srv = Server(ex, budget_bytes=8 << 30, n_slots=4, max_models=16)
    reqs = []
    for i, (key, op, x) in enumerate(specs):
        reqs.append(srv.submit(Request(i, key, op, x.shape[0], None, x)))
    for r in reqs:
        r.wait(120)
    srv.close()
    stats = dict(srv.sched.stats)
    note("server stats: %s" % stats)
    assert all(r.status == "done" for r in reqs), [(r.rid, r.status, r.error) for r in reqs]
    assert stats.get("batched_requests", 0) == len(reqs)
    ex.close()

    plans = {}
    for (key, op, x), r in zip(specs, reqs):
        if key not in plans:
            plans[key] = gf.plan(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, key.components, "f32")
        p = plans[key]
        xd = x.cuda()
        alone = (p.forward(xd) if op == "forward" else p.adjoint(xd)).cpu()
        got = r.result
        assert got.shape == alone.shape
        diff = float((got - alone).abs().max())
        assert diff == 0.0, (r.rid, op, diff)
    for p in plans.values():
        p.close()

    # one served forward against the oracle
    from synth import Geometry
    for (key, op, x), r in zip(specs, reqs):
        if op == "forward":
            g = Geometry(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h)
            st = np.array([(0, 0), (key.nx // 2, key.ny // 3), (key.nx - 1, key.ny - 1)])
            want = orc.forward(g, x[0].double().numpy(), st)
            got = r.result[0].double().numpy()
            comps = [c for c in range(7) if key.components >> c & 1]
            for i, c in enumerate(comps):
                gv = got[i][st[:, 1], st[:, 0]]
                e = np.linalg.norm(gv - want[:, c]) / np.linalg.norm(want[:, c])
                assert e <= 1e-5, (c, e)
            break
