"""Request loop (wfq_serve) on the GPU: each job's result is the same alone and in the mix, jobs
overlap on the device, the queue limit and unknown tickets are reported (needs an MI355X)."""

import time

import numpy as np
import pytest

from oracle import wfq_oracle as O
import wfq_inputs as wi
from wfq_inputs import geometry as geo
from helpers import GRAPHENE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2103_00438_amd import wfq
    wfq.load()
    return wfq


def jobs():
    out = []
    shapes = [geo.graphene_disk(14.0), geo.nanotube(5, 5, 30), geo.graphene_ribbon(12.0, 500),
              geo.graphene_disk(18.0), geo.nanotube(6, 6, 25), geo.graphene_ribbon(20.0, 700)]
    for k, xyz in enumerate(shapes):
        xyz = geo.jitter(xyz, 0.01, 300 + k)
        om = np.sort(0.05 + 0.95 * wi.uniform01(400 + k, 1 + (5 * k) % 7))
        dirs = np.eye(3)[: 1 + k % 3]
        out.append((xyz, om, dirs))
    return out


def test_mix_equals_alone(lib):
    tol = 1e-8
    js = jobs()
    srv = lib.wfq_serve(tol, max_jobs=3, max_queue=64, restart=40, precision="fp32")
    tickets = [lib.wfq_submit(srv, xyz, GRAPHENE, om, d) for xyz, om, d in js]
    results = [lib.wfq_wait(srv, t) for t in tickets]
    stats = lib.wfq_serve_stats(srv)
    lib.wfq_serve_stop(srv)
    assert stats["jobs_done"] == len(js)
    assert stats["max_resident"] >= 2                      # jobs overlapped on the device
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    for (xyz, om, d), res in zip(js, results):
        assert res["status"] == 0
        h = lib.wfq_build(xyz, GRAPHENE)
        alone = lib.wfq_solve(h, om, d, tol, restart=40, precision="fp32")
        h.close()
        err = np.linalg.norm(res["q"] - alone["q"]) / np.linalg.norm(alone["q"])
        assert err <= 1e-6
        assert all(i["relres"] <= tol for i in res["info"])
        assert res["timing"]["t_done_ms"] >= res["timing"]["t_admit_ms"] >= res["timing"]["t_submit_ms"]
    # one job against the oracle's dense solve
    xyz, om, d = js[0]
    P = O.Problem(xyz, GRAPHENE)
    q = results[0]["q"][0, 0]
    ref = P.solve_lu(om[0], d[0])
    assert np.linalg.norm(q - ref) / np.linalg.norm(ref) <= 1e-6


def test_mix_equals_alone_multishift(lib):
    # the request loop with one shared Krylov basis per job and direction (FP64 T)
    tol = 1e-8
    js = jobs()
    srv = lib.wfq_serve(tol, max_jobs=3, max_queue=64, restart=40, precision="fp64", algorithm="msgmres")
    tickets = [lib.wfq_submit(srv, xyz, GRAPHENE, om, d) for xyz, om, d in js]
    results = [lib.wfq_wait(srv, t) for t in tickets]
    lib.wfq_serve_stop(srv)
    for (xyz, om, d), res in zip(js, results):
        assert res["status"] == 0
        h = lib.wfq_build(xyz, GRAPHENE)
        alone = lib.wfq_solve(h, om, d, tol, restart=40, precision="fp64", algorithm="msgmres")
        batched = lib.wfq_solve(h, om, d, tol, restart=40, precision="fp64")
        h.close()
        assert np.linalg.norm(res["q"] - alone["q"]) / np.linalg.norm(alone["q"]) <= 1e-12   # deterministic
        assert np.linalg.norm(res["q"] - batched["q"]) / np.linalg.norm(batched["q"]) <= 1e-6
        assert all(i["relres"] <= tol for i in res["info"])


def test_queue_limit_and_tickets(lib):
    xyz, om, d = jobs()[3]
    srv = lib.wfq_serve(1e-8, max_jobs=1, max_queue=2, restart=40, precision="fp32")
    t = [lib.wfq_submit(srv, xyz, GRAPHENE, om, d)]
    time.sleep(0.0)
    codes = []
    for _ in range(4):
        try:
            t.append(lib.wfq_submit(srv, xyz, GRAPHENE, om, d))
        except lib.WfqError as e:
            codes.append(e.code)
    assert lib.WFQ_EAGAIN in codes
    with pytest.raises(lib.WfqError) as e:
        srv.jobs[987654] = (len(xyz), len(om), len(d))
        lib.wfq_poll(srv, 987654)
    assert e.value.code == lib.WFQ_ENOTFOUND
    for tk in t:
        assert lib.wfq_wait(srv, tk)["status"] == 0
    lib.wfq_serve_stop(srv)


def test_solve_dev_with_torch_buffers(lib):
    import torch
    xyz, om, d = jobs()[1]
    h = lib.wfq_build(xyz, GRAPHENE)
    host = lib.wfq_solve(h, om, d, 1e-9, restart=40, precision="fp32")
    dev = torch.device("cuda:0")
    S, n = len(om) * len(d), len(xyz)
    qr = torch.zeros(S * n, dtype=torch.float64, device=dev)
    qi = torch.zeros(S * n, dtype=torch.float64, device=dev)
    ar = torch.zeros(S * 3, dtype=torch.float64, device=dev)
    ai = torch.zeros(S * 3, dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(dev)
    out = lib.wfq_solve_dev(h, om, d, 1e-9, q_re=qr, q_im=qi, alpha_re=ar, alpha_im=ai,
                            stream=stream.cuda_stream, restart=40, precision="fp32")
    torch.cuda.synchronize()
    q = (qr.cpu().numpy() + 1j * qi.cpu().numpy()).reshape(len(om), len(d), n)
    a = (ar.cpu().numpy() + 1j * ai.cpu().numpy()).reshape(len(om), len(d), 3)
    assert out["status"] == 0
    assert np.array_equal(q, host["q"])            # same kernels, same order: bit-identical
    assert np.array_equal(a, host["alpha"])
    h.close()
