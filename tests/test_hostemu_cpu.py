"""The GPU wave operators (ops64.h), run lane by lane on the CPU by the host
emulation harness, against numpy's FFT and the FP64 oracle.

This checks the index logic of the transforms the kernels use -- the same
source code -- without a GPU.
"""

import ctypes
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.environ.get("MOMFBD_HOSTEMU") or os.path.join(os.path.dirname(HERE),
                                                        "paper_2505_10639_amd",
                                                        "libmomfbd_hostemu.so")
FP = ctypes.POINTER(ctypes.c_float)


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        pytest.fail("libmomfbd_hostemu.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(EMU)


def ptr(a):
    return a.ctypes.data_as(FP)


def rng(k):
    return np.random.default_rng(500 + k)


@pytest.mark.parametrize("L,d", [(32, -1), (32, 1), (64, -1), (64, 1)])
def test_in_lane_fft(emu, L, d):
    x = (rng(L).standard_normal(L) + 1j * rng(L + 1).standard_normal(L)).astype(np.complex64)
    y = x.copy()
    (emu.emu_fft32 if L == 32 else emu.emu_fft64)(ptr(y.view(np.float32)), d)
    ref = np.fft.fft(x.astype(complex)) if d < 0 else np.fft.ifft(x.astype(complex)) * L
    assert np.abs(y - ref).max() <= 3e-7 * np.abs(ref).max()


def test_real_forward_2d(emu):
    img = rng(1).standard_normal((64, 64)).astype(np.float32)
    half = np.zeros((64, 33), np.complex64)
    emu.emu_r2c(ptr(img), ptr(half.view(np.float32)))
    ref = oracle.dft2(img)[:, :33]
    assert np.abs(half - ref).max() <= 5e-7 * np.abs(ref).max()


def test_real_forward_2d_half_buffer(emu):
    """The forward kernel's form: transposes through a half-size buffer,
    real parts then imaginary parts."""
    img = rng(11).standard_normal((64, 64)).astype(np.float32)
    half = np.zeros((64, 33), np.complex64)
    emu.emu_r2c_half(ptr(img), ptr(half.view(np.float32)))
    ref = oracle.dft2(img)[:, :33]
    assert np.abs(half - ref).max() <= 5e-7 * np.abs(ref).max()


def test_band_pupil_inverse_half_buffer(emu):
    A = synth.pupil_mask(64)[16:48, 16:48].astype(np.float32)
    ph = (0.2 * rng(13).standard_normal((32, 32))).astype(np.float32)
    p = np.zeros((64, 64), np.complex64)
    emu.emu_pupil_ifft_half(ptr(A), ptr(ph), ptr(p.view(np.float32)))
    P = np.zeros((64, 64), complex)
    P[16:48, 16:48] = A * np.exp(2j * np.pi * ph.astype(np.float64))
    ref = oracle.idft2_un(P)
    assert np.abs(p - ref).max() <= 5e-7 * np.abs(ref).max()


def test_hermitian_inverse_2d(emu):
    H = oracle.dft2(rng(2).standard_normal((64, 64)))
    half = H[:, :33].astype(np.complex64)
    out = np.zeros((64, 64), np.float32)
    emu.emu_c2r(ptr(half.view(np.float32)), ptr(out))
    ref = oracle.idft2_un(oracle.expand_half(half, 64)).real
    assert np.abs(out - ref).max() <= 5e-7 * np.abs(ref).max()


def test_band_pupil_inverse(emu):
    A = synth.pupil_mask(64)[16:48, 16:48].astype(np.float32)
    ph = (0.2 * rng(3).standard_normal((32, 32))).astype(np.float32)
    p = np.zeros((64, 64), np.complex64)
    emu.emu_pupil_ifft(ptr(A), ptr(ph), ptr(p.view(np.float32)))
    P = np.zeros((64, 64), complex)
    P[16:48, 16:48] = A * np.exp(2j * np.pi * ph.astype(np.float64))
    ref = oracle.idft2_un(P)
    assert np.abs(p - ref).max() <= 5e-7 * np.abs(ref).max()


def test_forward_on_band(emu):
    h = (rng(4).standard_normal((64, 64)) + 1j * rng(5).standard_normal((64, 64))).astype(np.complex64)
    band = np.zeros((32, 32), np.complex64)
    emu.emu_fft_to_band(ptr(h.view(np.float32)), ptr(band.view(np.float32)))
    ref = oracle.dft2(h)[16:48, 16:48]
    assert np.abs(band - ref).max() <= 5e-7 * np.abs(ref).max()


def test_unit_chain_matches_oracle_gradient(emu):
    """PSF, OTF and dL/dphi of one unit against the oracle's formulas."""
    pr = synth.make_problem(31, N=64, P=1, J=1, M=20, d_over_r0=12.0)
    A = pr.pupil[0].astype(np.float64)
    phi = oracle.wavefront(pr.alpha_true[0, 0], pr.basis[0], pr.diversity[0])
    Ab = A[16:48, 16:48].astype(np.float32)
    ph = (phi[16:48, 16:48] / (2 * np.pi)).astype(np.float32)
    kap = 1.0 / (64 * 64 * A.sum())
    G = oracle.dft2(rng(6).standard_normal((64, 64)))      # any Hermitian spectrum
    Gh = G[:, :33].astype(np.complex64)
    psf = np.zeros((64, 64), np.float32)
    S = np.zeros((64, 33), np.complex64)
    gphi = np.zeros((32, 32), np.float32)
    emu.emu_unit(ptr(Ab), ptr(ph), ctypes.c_float(kap), ptr(Gh.view(np.float32)), ptr(psf),
                 ptr(S.view(np.float32)), ptr(gphi))
    P = oracle.pupil_field(A, phi)
    p = oracle.psf_field(P)
    s = kap * np.abs(p) ** 2
    assert np.abs(psf - s).max() <= 1e-6 * s.max()
    S_ref = oracle.otf(s)[:, :33]
    assert np.abs(S - S_ref).max() <= 1e-6
    g_s = oracle.idft2_un(oracle.expand_half(Gh, 64)).real
    GP = oracle.dft2(2 * kap * g_s * p)
    ref = (np.conj(P) * GP).imag[16:48, 16:48]
    assert np.abs(gphi - ref).max() <= 2e-5 * np.abs(ref).max()


def test_fused_adjoint_path_matches_unfused(emu):
    """The register-saving fused adjoint (op14) gives the same dL/dphi."""
    pr = synth.make_problem(32, N=64, P=1, J=1, M=20, d_over_r0=12.0)
    A = pr.pupil[0].astype(np.float64)
    phi = oracle.wavefront(pr.alpha_true[0, 0], pr.basis[0], pr.diversity[0])
    Ab = A[16:48, 16:48].astype(np.float32)
    ph = (phi[16:48, 16:48] / (2 * np.pi)).astype(np.float32)
    kap = 1.0 / (64 * 64 * A.sum())
    Gh = oracle.dft2(rng(7).standard_normal((64, 64)))[:, :33].astype(np.complex64)
    g1 = np.zeros((32, 32), np.float32)
    g2 = np.zeros((32, 32), np.float32)
    psf = np.zeros((64, 64), np.float32)
    S = np.zeros((64, 33), np.complex64)
    emu.emu_unit(ptr(Ab), ptr(ph), ctypes.c_float(kap), ptr(Gh.view(np.float32)), ptr(psf),
                 ptr(S.view(np.float32)), ptr(g1))
    emu.emu_unit_fused(ptr(Ab), ptr(ph), ctypes.c_float(kap), ptr(Gh.view(np.float32)), ptr(g2))
    P = oracle.pupil_field(A, phi)
    g_s = oracle.idft2_un(oracle.expand_half(Gh, 64)).real
    ref = (np.conj(P) * oracle.dft2(2 * kap * g_s * oracle.psf_field(P))).imag[16:48, 16:48]
    assert np.abs(g2 - ref).max() <= 2e-5 * np.abs(ref).max()
    assert np.abs(g2 - g1).max() <= 2e-5 * np.abs(ref).max()


# ----------------------------------------------------------------- N = 128

def test_n128_band_pupil_inverse(emu):
    A = synth.pupil_mask(128)[32:96, 32:96].astype(np.float32)
    ph = (0.2 * rng(11).standard_normal((64, 64))).astype(np.float32)
    p = np.zeros((128, 128), np.complex64)
    emu.emu128_pupil_ifft(ptr(A), ptr(ph), ptr(p.view(np.float32)))
    P = np.zeros((128, 128), complex)
    P[32:96, 32:96] = A * np.exp(2j * np.pi * ph.astype(np.float64))
    ref = oracle.idft2_un(P)
    assert np.abs(p - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n128_real_forward(emu):
    img = rng(12).standard_normal((128, 128)).astype(np.float32)
    half = np.zeros((128, 65), np.complex64)
    emu.emu128_r2c(ptr(img), ptr(half.view(np.float32)))
    ref = oracle.dft2(img)[:, :65]
    assert np.abs(half - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n128_band_pupil_inverse_half_buffer(emu):
    """The forward kernel's form at 128: both transposes through a half-size
    buffer, real parts then imaginary parts."""
    A = synth.pupil_mask(128)[32:96, 32:96].astype(np.float32)
    ph = (0.2 * rng(16).standard_normal((64, 64))).astype(np.float32)
    p = np.zeros((128, 128), np.complex64)
    emu.emu128_pupil_ifft_half(ptr(A), ptr(ph), ptr(p.view(np.float32)))
    P = np.zeros((128, 128), complex)
    P[32:96, 32:96] = A * np.exp(2j * np.pi * ph.astype(np.float64))
    ref = oracle.idft2_un(P)
    assert np.abs(p - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n128_real_forward_half_buffer(emu):
    img = rng(17).standard_normal((128, 128)).astype(np.float32)
    half = np.zeros((128, 65), np.complex64)
    emu.emu128_r2c_half(ptr(img), ptr(half.view(np.float32)))
    ref = oracle.dft2(img)[:, :65]
    assert np.abs(half - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n128_hermitian_inverse(emu):
    H = oracle.dft2(rng(13).standard_normal((128, 128)))
    half = H[:, :65].astype(np.complex64)
    out = np.zeros((128, 128), np.float32)
    emu.emu128_c2r(ptr(half.view(np.float32)), ptr(out))
    ref = oracle.idft2_un(oracle.expand_half(half, 128)).real
    assert np.abs(out - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n128_forward_on_band(emu):
    h = (rng(14).standard_normal((128, 128)) + 1j * rng(15).standard_normal((128, 128))).astype(np.complex64)
    band = np.zeros((64, 64), np.complex64)
    emu.emu128_fft_to_band(ptr(h.view(np.float32)), ptr(band.view(np.float32)))
    ref = oracle.dft2(h)[32:96, 32:96]
    assert np.abs(band - ref).max() <= 5e-7 * np.abs(ref).max()


# ------------------------------------------------------------------ N = 96

@pytest.mark.parametrize("d", [-1, 1])
def test_n96_fft48(emu, d):
    x = (rng(20).standard_normal(48) + 1j * rng(21).standard_normal(48)).astype(np.complex64)
    y = x.copy()
    emu.emu96_fft48(ptr(y.view(np.float32)), d)
    ref = np.fft.fft(x.astype(complex)) if d < 0 else np.fft.ifft(x.astype(complex)) * 48
    assert np.abs(y - ref).max() <= 3e-7 * np.abs(ref).max()


def test_n96_band_pupil_inverse(emu):
    A = synth.pupil_mask(96)[24:72, 24:72].astype(np.float32)
    ph = (0.2 * rng(22).standard_normal((48, 48))).astype(np.float32)
    p = np.zeros((96, 96), np.complex64)
    emu.emu96_pupil_ifft(ptr(A), ptr(ph), ptr(p.view(np.float32)))
    P = np.zeros((96, 96), complex)
    P[24:72, 24:72] = A * np.exp(2j * np.pi * ph.astype(np.float64))
    ref = oracle.idft2_un(P)
    assert np.abs(p - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n96_real_forward_and_inverse(emu):
    img = rng(23).standard_normal((96, 96)).astype(np.float32)
    half = np.zeros((96, 49), np.complex64)
    emu.emu96_r2c(ptr(img), ptr(half.view(np.float32)))
    ref = oracle.dft2(img)[:, :49]
    assert np.abs(half - ref).max() <= 5e-7 * np.abs(ref).max()
    H = oracle.dft2(rng(24).standard_normal((96, 96)))
    hh = H[:, :49].astype(np.complex64)
    out = np.zeros((96, 96), np.float32)
    emu.emu96_c2r(ptr(hh.view(np.float32)), ptr(out))
    ref = oracle.idft2_un(oracle.expand_half(hh, 96)).real
    assert np.abs(out - ref).max() <= 5e-7 * np.abs(ref).max()


def test_n96_unit_chain_matches_oracle_gradient(emu):
    pr = synth.make_problem(33, N=96, P=1, J=1, M=20, d_over_r0=12.0)
    A = pr.pupil[0].astype(np.float64)
    phi = oracle.wavefront(pr.alpha_true[0, 0], pr.basis[0], pr.diversity[0])
    Ab = A[24:72, 24:72].astype(np.float32)
    ph = (phi[24:72, 24:72] / (2 * np.pi)).astype(np.float32)
    kap = 1.0 / (96 * 96 * A.sum())
    Gh = oracle.dft2(rng(25).standard_normal((96, 96)))[:, :49].astype(np.complex64)
    psf = np.zeros((96, 96), np.float32)
    S = np.zeros((96, 49), np.complex64)
    gphi = np.zeros((48, 48), np.float32)
    emu.emu96_unit(ptr(Ab), ptr(ph), ctypes.c_float(kap), ptr(Gh.view(np.float32)), ptr(psf),
                   ptr(S.view(np.float32)), ptr(gphi))
    P = oracle.pupil_field(A, phi)
    p = oracle.psf_field(P)
    s = kap * np.abs(p) ** 2
    assert np.abs(psf - s).max() <= 1e-6 * s.max()
    assert np.abs(S - oracle.otf(s)[:, :49]).max() <= 1e-6
    g_s = oracle.idft2_un(oracle.expand_half(Gh, 96)).real
    ref = (np.conj(P) * oracle.dft2(2 * kap * g_s * p)).imag[24:72, 24:72]
    assert np.abs(gphi - ref).max() <= 2e-5 * np.abs(ref).max()


# ------------------------------------------------ bf16 split of FP32 values
def _split3(emu, x):
    x = np.ascontiguousarray(x, np.float32)
    parts = np.zeros((x.size, 3), np.float32)
    emu.emu_split3(ptr(x), ctypes.c_int(x.size), ptr(parts))
    return parts


def _split_inputs():
    r = rng(40)
    mags = 2.0 ** r.integers(-100, 100, 4000)
    x = (r.standard_normal(4000) * mags).astype(np.float32)
    # exact for 0 and |x| >= 2^-110 (below, the bits under 2^-133 are lost)
    special = np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 2.0 ** -110, -(2.0 ** -110),
                        1.1754944e-38, np.float32(1) + np.float32(2 ** -23), 65504.0, 1.0 / 3.0],
                       np.float32)
    return np.concatenate([x, special])


def test_bf16_split_is_exact(emu):
    """hi + mid + lo equals x exactly and every part is a bf16 (low 16 bits
    zero): the contractions' operands lose nothing in the split."""
    x = _split_inputs()
    p = _split3(emu, x)
    assert np.all((p.view(np.uint32) & 0xFFFF) == 0)
    assert np.array_equal(p.astype(np.float64).sum(1), x.astype(np.float64))
    # the parts shrink by at least 2^7 and 2^15 relative to |x|
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(p[:, 1]) <= ax * 2.0 ** -7)
    assert np.all(np.abs(p[:, 2]) <= ax * 2.0 ** -15)


def test_six_partial_products_keep_fp32_accuracy(emu):
    """The six products with part orders adding to at most 2 reproduce x y
    within 2^-21 |x y| (the bound the contraction code states)."""
    r = rng(41)
    x = (r.standard_normal(5000) * 2.0 ** r.integers(-20, 20, 5000)).astype(np.float32)
    y = (r.standard_normal(5000) * 2.0 ** r.integers(-20, 20, 5000)).astype(np.float32)
    a, b = _split3(emu, x).astype(np.float64), _split3(emu, y).astype(np.float64)
    six = (a[:, 0] * b[:, 0] + a[:, 0] * b[:, 1] + a[:, 1] * b[:, 0] + a[:, 0] * b[:, 2]
           + a[:, 2] * b[:, 0] + a[:, 1] * b[:, 1])
    exact = x.astype(np.float64) * y.astype(np.float64)
    assert np.all(np.abs(six - exact) <= 2.0 ** -21 * np.abs(exact))


@pytest.mark.parametrize("tiny", [False, True])
def test_bf16_split_packing(emu, tiny):
    """Eight values pack two per word, element e in bits 16 (e & 1) of word
    e >> 1, one group of four words per part.  Values below 2^-110 (which a
    basis holds as rounding noise where a mode vanishes) leave their packed
    neighbours intact."""
    x = (rng(42).standard_normal(8) * 10).astype(np.float32)
    if tiny:
        x[1], x[4], x[7] = -8.803836e-35, 1.3159354e-33, 3e-38
    words = np.zeros(12, np.uint32)
    emu.emu_split8(ptr(x), words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    p = _split3(emu, x).view(np.uint32)
    assert np.all((p & 0xFFFF) == 0)
    for part in range(3):
        w = words[4 * part:4 * part + 4]
        got = np.stack([w & 0xFFFF, w >> 16], 1).reshape(8)
        assert np.array_equal(got, p[:, part] >> 16)
    # the parts of the values of normal size still add up to them exactly
    ok = np.abs(x.astype(np.float64)) >= 2.0 ** -110
    assert np.array_equal(p.view(np.float32).astype(np.float64).sum(1)[ok], x.astype(np.float64)[ok])
