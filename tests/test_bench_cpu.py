"""Host logic of bench.py: the counted-traffic lookup, the roofline object
and the one-GPU guard (no GPU needed)."""

import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counted_traffic_follows_schedule(bench):
    sched = {"xcd_forward": 0, "xcd_adjoint": 1, "object_pairs_per_thread": 1, "grad_waves": 4}
    for (kern, N), rec in bench.COUNTED_TRAFFIC.items():
        if rec["sources_sha1"] != bench.sources_sha(kern, N):
            assert bench.counted_traffic(kern, sched, N) is None
            continue
        for v, (rd, wr) in rec["by_value"].items():
            assert bench.counted_traffic(kern, dict(sched, **{rec["knob"]: v}), N) == rd + wr
        # a knob value the counters were not taken for reports nothing
        assert bench.counted_traffic(kern, dict(sched, **{rec["knob"]: 99}), N) is None
    assert bench.counted_traffic("no_such_kernel", sched) is None
    assert bench.counted_traffic("adjoint", sched, 96) is None


def test_counted_traffic_stale_source(bench, monkeypatch):
    key = ("adjoint", 64)
    monkeypatch.setitem(bench.COUNTED_TRAFFIC, key,
                        dict(bench.COUNTED_TRAFFIC[key], sources_sha1="000000000000"))
    assert bench.counted_traffic("adjoint", {"xcd_adjoint": 1}) is None


def test_roofline_alu_and_hbm(bench):
    N, P, J, units = 64, 10, 12, 240
    chan_obj, frac = [0, 1], [0.5, 0.25]
    _, per_kernel = bench.unit_flops(N)
    unit = N * 33 * 8
    nb = bench.kernel_io_bytes(N, P, J, chan_obj, frac)
    # adjoint: D, S (one channel per object here) and O within the support,
    # phi read and dL/dphi written on the 32 x 32 band
    spec_in = P * J * unit * (0.5 + 0.25)
    assert nb["adjoint"] == pytest.approx(2 * spec_in + P * unit * 0.75 + 2 * units * 1024 * 4)
    assert nb["forward"] == units * 1024 * 4 + units * unit
    assert nb["object"] == pytest.approx(units * unit + spec_in + P * 2 * unit)
    r = bench.roofline({"adjoint": 2.0, "forward": 1.0}, units, N, nb, lambda k: 123)
    assert r["kernel"] == "adjoint" and r["bound"] == "alu" and r["traffic"] == 123
    assert r["achieved"] == pytest.approx(per_kernel["adjoint"] * units / 2e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    hv = r["hbm_view"]
    assert hv["achieved"] == pytest.approx(nb["adjoint"] / 2e-3 / 1e9)
    assert hv["frac"] == pytest.approx(hv["achieved"] / 8000.0)
    r = bench.roofline({"object": 4.0, "adjoint": 1.0}, units, N, nb, lambda k: None)
    assert r["bound"] == "hbm" and r["traffic"] is None and "hbm_view" not in r
    assert r["achieved"] == pytest.approx(nb["object"] / 4e-3 / 1e9)


def test_support_fraction(bench):
    """The bench's support rule against the exact OTF support (where the
    pupil autocorrelation is nonzero): equal for a disk, a superset for two
    separate sub-apertures."""
    import synth
    N = 64
    y, x = np.mgrid[0:N, 0:N]
    two = (((y - 31) ** 2 + (x - 23) ** 2 <= 25) | ((y - 33) ** 2 + (x - 41) ** 2 <= 25))
    for A, exact_match in ((synth.pupil_mask(N, 0.45) > 0, True), (two, False)):
        ac = np.real(np.fft.ifft2(np.abs(np.fft.fft2(A.astype(float))) ** 2))
        exact = float(np.mean(ac[:, : N // 2 + 1] > 0.5))
        f = bench.support_fraction([A], [0], N)[0]
        assert f >= exact
        if exact_match:
            assert f == pytest.approx(exact)
    # the 0.45 N disk: 62.4% of the half spectrum
    assert bench.support_fraction([synth.pupil_mask(N, 0.45) > 0], [0], N)[0] == \
        pytest.approx(1317 / 2112)


def test_fft_flop_count(bench):
    # 5 N^2 log2(N^2) for a complex N x N transform; the real one half of it
    c2c, real = bench.fft_flops(64)
    assert c2c == pytest.approx(5 * 64 * 64 * 12) and real == pytest.approx(c2c / 2)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in p.stdout + p.stderr
