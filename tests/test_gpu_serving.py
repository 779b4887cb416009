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
    for i in range(16):
        n = int(rng.choice([64, 128]))
        nz = int(rng.choice([8, 16]))
        # gz, the six stored components, all nine (two column-pass groups),
        # gz with the first derivatives
        comps = int(rng.choice([0x3F, 0x1, 0x1FF, 0x181]))
        op = "forward" if rng.random() < 0.5 else "adjoint"
        B = int(rng.integers(1, 5))
        # some geometries are layered meshes (thickening layers, buried top)
        # some geometries are layered meshes, some have three observation levels
        zedges, levels = None, 1
        u = rng.random()
        if u < 0.25:
            zedges = tuple(float(v) for v in 5.0 + np.concatenate([[0.0], np.cumsum(6.0 * 1.2 ** np.arange(nz))]))
        elif u < 0.5:
            levels = 3
        key = GeometryKey(n, n, nz, 20.0, 20.0, 20.0, 10.0, comps, zedges, levels)
        shape = (B, nz, n, n) if op == "forward" else (B,) + key.data_shape
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
    # device-side times of each request's group: copies and operator within
    # the request's wall-clock latency
    for r in reqs:
        assert r.device_ms is not None and r.compute_ms is not None, r.rid
        assert 0.0 < r.compute_ms <= r.device_ms <= r.latency * 1e3 + 1.0, (r.rid, r.compute_ms, r.device_ms)
    ex.close()

    plans = {}
    for (key, op, x), r in zip(specs, reqs):
        if key not in plans:
            if key.levels > 1:
                plans[key] = gf.plan_levels(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, key.levels,
                                            key.components, "f32")
            elif key.zedges is None:
                plans[key] = gf.plan(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, key.components, "f32")
            else:
                plans[key] = gf.plan_layered(key.nx, key.ny, key.dx, key.dy, key.zedges, key.h, key.components,
                                             "f32")
        p = plans[key]
        xd = x.cuda()
        alone = (p.forward(xd) if op == "forward" else p.adjoint(xd)).cpu()
        got = r.result
        assert got.shape == alone.shape
        diff = float((got - alone).abs().max())
        assert diff == 0.0, (r.rid, op, diff)
    for p in plans.values():
        p.close()

    # served forwards against the oracle: the first uniform and the first
    # layered one
    from synth import Geometry
    seen = set()
    for (key, op, x), r in zip(specs, reqs):
        kind = (key.zedges is not None, key.levels)
        if op == "forward" and kind not in seen:
            seen.add(kind)
            g = Geometry(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h)
            st = np.array([(0, 0), (key.nx // 2, key.ny // 3), (key.nx - 1, key.ny - 1)])
            if key.levels > 1:
                want_l = orc.forward_levels(g, x[0].double().numpy(), key.levels, st)
                got_l = r.result[0].double().numpy()
            else:
                want_l = orc.forward(g, x[0].double().numpy(), st, zedges=key.zedges)[None]
                got_l = r.result[0].double().numpy()[None]
            comps = [c for c in range(9) if key.components >> c & 1]
            for t in range(want_l.shape[0]):
                for i, c in enumerate(comps):
                    gv = got_l[t][i][st[:, 1], st[:, 0]]
                    e = np.linalg.norm(gv - want_l[t][:, c]) / np.linalg.norm(want_l[t][:, c])
                    assert e <= 1e-5, (key, t, c, e)
    assert seen, "no served forward to check"


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_workspace_estimate_bounds_the_plan(gf, prec):
    """Admission sizes a request's workspace before its plan exists; that
    estimate must not fall below what the plan then asks for."""
    from paper_2005_10160_amd.serve import GeometryKey, GpuExecutor
    ex = GpuExecutor(prec, 1)
    cases = [(64, 8, 0x1), (64, 8, 0x1FF), (100, 37, 0x1FF), (128, 16, 0x3F), (33, 5, 0x181), (96, 3, 0x7F),
             (140, 9, 0x1), (140, 9, 0x41)]
    for n, nz, comps in cases:
        for zedges, levels in ((None, 1), (tuple(float(v) for v in np.cumsum(np.r_[0.0, 3.0 * 1.3 ** np.arange(nz)])), 1),
                               (None, 3), (None, 11)):
            key = GeometryKey(n, n + 7, nz, 20.0, 20.0, 20.0, 10.0, comps, zedges, levels)
            est = {(op, B): ex.workspace_bytes(key, op, B) for op in ("forward", "adjoint") for B in (1, 3, 16)}
            if levels > 1:
                p = gf.plan_levels(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, levels, comps, prec)
            elif zedges is None:
                p = gf.plan(key.nx, key.ny, key.nz, key.dx, key.dy, key.dz, key.h, comps, prec)
            else:
                p = gf.plan_layered(key.nx, key.ny, key.dx, key.dy, zedges, key.h, comps, prec)
            for (op, B), e in est.items():
                need = p.workspace_bytes(op, B)
                assert need <= e, (key, op, B, need, e)
            p.close()
    ex.close()
