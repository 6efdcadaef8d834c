"""The library's counter-based normal generator against the reference:
the generator words bit for bit, the normals to FP32 rounding."""

import numpy as np
import pytest

from oracle import rng

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2505_10639_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("seed,sid,c0,n", [(0, 0, 0, 4096), (0xDEADBEEF12345678, 5, 1 << 33, 1001),
                                           (7, (1 << 40) + 3, 123, 3)])
def test_words_and_normals_match_reference(dev, seed, sid, c0, n):
    from paper_2505_10639_amd import _lib
    out = torch.empty(n, dtype=torch.float32, device=dev)
    bits = torch.empty(n, dtype=torch.int32, device=dev)
    _lib.momfbd_random_normal(seed, sid, c0, out, bits)
    torch.cuda.synchronize()
    w = bits.cpu().numpy().view(np.uint32)
    assert np.array_equal(w, rng.words(seed, sid, c0, n))
    z = out.cpu().numpy().astype(np.float64)
    ref = rng.normals(seed, sid, c0, n)
    assert np.all(np.abs(z - ref) <= 2e-6 * (1.0 + np.abs(ref)))


def test_calls_continue_one_another(dev):
    from paper_2505_10639_amd import _lib
    a = torch.empty(4000, dtype=torch.float32, device=dev)
    b = torch.empty(1000, dtype=torch.float32, device=dev)
    c = torch.empty(3000, dtype=torch.float32, device=dev)
    _lib.momfbd_random_normal(11, 2, 0, a)
    _lib.momfbd_random_normal(11, 2, 0, b)
    _lib.momfbd_random_normal(11, 2, 250, c)
    torch.cuda.synchronize()
    assert torch.equal(a[:1000], b) and torch.equal(a[1000:], c)
    big = torch.empty(1 << 22, dtype=torch.float32, device=dev)
    _lib.momfbd_random_normal(3, 0, 0, big)
    zs = big.double()
    assert abs(float(zs.mean())) < 4.0 / 2048 and abs(float(zs.std()) - 1.0) < 3e-3
