"""twa_run_noalloc (the entry point for callers that cannot allocate device
memory: every buffer in the library's fixed device scratch array) through the
C ABI against twa_run on the same inputs, bit for bit: two calls in a row,
the second with a smaller input (the array keeps the first call's contents),
on the multi-kernel path (FP32, BF16, semi-implicit) and the fused small-N
path (FP64); plus the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KEYS = ("T2", "T3", "T4", "Z", "ZZ", "Sz", "SpSm", "g2", "T2_se", "SpSm_se", "g2_se", "max_norm_dev", "n_samples",
        "tile_config", "nan_flag", "step_criterion")


@pytest.fixture(scope="module")
def twa():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_10075_amd as m
    return m


def _same(a, b):
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])


@pytest.mark.parametrize("prec,integ", [("fp32", "heun"), ("bf16", "sib"), ("fp64", "heun")])
def test_noalloc_equals_twa_run_twice_shrinking(twa, prec, integ):
    cases = [(300, 2.0, 1.0, 256, 120, 5), (70, 1.0, 0.5, 48, 80, 9)]   # (N, w, alpha, B, T, seed)
    for N, w, a, B, T, seed in cases:
        p = twa.build_pump(N, w, a)
        dt = 0.02 / N
        print("noalloc %s %s N=%d B=%d T=%d" % (prec, integ, N, B, T), flush=True)
        got = twa.run_noalloc(p, B, dt, T, seed=seed, precision=prec, integrator=integ, norm_tol=-1)
        ref = twa.run(p, B, dt, T, seed=seed, precision=prec, integrator=integ, norm_tol=-1, use_graph=False).obs
        _same(got, ref)


def test_noalloc_fused_small_n(twa):
    for N, B in ((16, 512), (9, 40)):
        p = twa.build_pump(N, 4.0, 1.0)
        got = twa.run_noalloc(p, B, 1e-3, 300, seed=1, precision="fp64", s0z=-1.0, norm_tol=-1)
        ref = twa.run(p, B, 1e-3, 300, seed=1, precision="fp64", s0z=-1.0, norm_tol=-1).obs
        assert got["tile_config"] == 99
        _same(got, ref)


def test_noalloc_rejects_what_it_cannot_hold(twa):
    p = twa.build_pump(3000, 1.0, 1.0)
    with pytest.raises(twa.TWAError) as e:
        twa.run_noalloc(p, 4096, 1e-4, 10, precision="fp32")
    assert e.value.code == twa.TWA_ENOMEM and "scratch" in str(e.value)
    q = twa.build_pump(20, 1.0, 1.0)
    with pytest.raises(twa.TWAError) as e:
        twa.run_noalloc(q, 8, 1e-3, 10, burnin=10)
    assert e.value.code == twa.TWA_EINVAL
