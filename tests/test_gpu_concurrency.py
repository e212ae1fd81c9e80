"""Library calls from several host threads at once: single runs that capture
and replay hipGraphs on their own streams (torch streams and streams the
library creates), a batched scan and pump builds (rocSOLVER).  The library
serialises its entry points (hipFree synchronises the whole device, which
must not happen inside another call's graph capture), so no call may fail,
and every result must equal the same call made alone, bit for bit."""
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def test_threads_do_not_disturb_each_others_graph_capture(twa):
    import torch
    N, B, T, dt = 300, 64, 200, 5e-5          # 200 steps: 12 graph captures per run
    pump = twa.build_pump(N, 2.0, 1.0)
    kw = dict(precision="fp32", norm_tol=-1)
    pts = [(70, 1.0, 0.5, 2e-4, 11), (300, 2.0, 1.0, 6e-5, 12)]
    seeds = [1, 2, 3]
    ref = [twa.run(pump, B, dt, T, seed=s, **kw).obs for s in seeds]
    ref_batch = twa.run_batch(pts, 32, 120, **kw)
    ref_lam = twa.build_pump(130, 1.5, 0.5).lam_max
    rng = np.random.default_rng(4)
    M = rng.standard_normal((40, 40))
    dense = M @ M.T / 40.0
    ref_dense = twa.Pump(40, dense=dense).matrix("F")

    streams = [torch.cuda.Stream(), torch.cuda.Stream(), None]
    out, batch_out, lams, dense_out, errors = [None] * 3, [], [], [], []

    def single(i):
        try:
            for _ in range(3):
                out[i] = twa.run(pump, B, dt, T, seed=seeds[i], stream=streams[i], **kw).obs
        except Exception as e:   # collected and asserted on the main thread
            errors.append("run %d: %r" % (i, e))

    def batch():
        try:
            for _ in range(3):
                batch_out.append(twa.run_batch(pts, 32, 120, **kw))
        except Exception as e:
            errors.append("batch: %r" % e)

    def builds():
        try:
            for _ in range(3):
                q = twa.build_pump(130, 1.5, 0.5)
                lams.append(q.lam_max)
                q.close()
                d = twa.Pump(40, dense=dense)
                dense_out.append(d.matrix("F"))
                d.close()
        except Exception as e:
            errors.append("pump build: %r" % e)

    threads = [threading.Thread(target=single, args=(i,)) for i in range(3)]
    threads += [threading.Thread(target=batch), threading.Thread(target=builds)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in threads), "a thread did not finish"
    assert not errors, errors
    for i in range(3):
        for k in ("SpSm", "g2", "Sz", "T2", "ZZ", "max_norm_dev"):
            assert out[i][k] == ref[i][k], (i, k)
    assert len(batch_out) == 3
    for res in batch_out:
        for a, b in zip(res, ref_batch):
            assert a["g2"] == b["g2"] and a["SpSm"] == b["SpSm"]
    # (the eigensolver is not promised to be bitwise repeatable)
    assert len(lams) == 3 and all(abs(x - ref_lam) <= 1e-12 * abs(ref_lam) for x in lams)
    assert len(dense_out) == 3
    for F in dense_out:
        assert np.max(np.abs(F - ref_dense)) <= 1e-12 * np.max(np.abs(ref_dense))
