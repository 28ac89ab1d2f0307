"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test compares the vectorised oracle with something it does not share code with: pure-Python direct
sums of Eq. (1)-(3)/(5), a closed form (the correlogram at alpha = 0, the Welch sum), an algebraic identity
(conjugate symmetry, scale, linearity), or a property the paper states for its test signals (cycle
frequencies of BPSK and of DSSS BPSK).
"""
import json
import os

import numpy as np
import pytest

from oracle import brute as B
from oracle import scd_oracle as O
from synth import signals as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sig(n, seed, kind="bpsk"):
    rng = sg.rng_for(90, seed)
    if kind == "bpsk":
        return sg.bpsk(n, 0.07, 4, 3.0, rng)
    return sg.noise(n, rng)


@pytest.mark.parametrize("N,Np,kind", [(64, 8, "bpsk"), (32, 16, "noise")])
def test_ssca_equals_eq2_direct_sum(N, Np, kind):
    """Every SSCA cell equals the Eq. (2) correlation of two Eq. (1) demodulates (pins framing, padding,
    down-conversion sign and phase, the k and q orders and the (f, alpha) map together)."""
    x = _sig(N, 1, kind)
    w = sg.hamming(Np)
    S = O.ssca(x, Np, w)
    xs, ws = list(x), list(w)
    ref = np.array([[B.ssca_cell_eq2(xs, ws, k, q) for q in range(N)] for k in range(Np)])
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("conjugate", [False, True])
def test_ssca_cross_equals_eq2_direct_sum(conjugate):
    """Cross and conjugate SSCA cells equal Eq. (2) with a second input y (y != x, both complex): pins which
    operand is conjugated and the sign of y's frequency."""
    N, Np = 32, 8
    x, y = _sig(N, 3, "noise"), _sig(N, 4, "noise")
    w = sg.hamming(Np)
    S = O.ssca_cross(x, y, Np, w, conjugate)
    ref = np.array([[B.ssca_cross_cell_eq2(list(x), list(y), list(w), k, q, conjugate) for q in range(N)]
                    for k in range(Np)])
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ssca_cross_special_cases():
    """y = x gives the auto SCD exactly; for a real x the conjugate form equals the auto SCD too; swapping the
    roles of x and y changes the result (the cross form is not symmetric in its inputs)."""
    N, Np = 256, 16
    x, y = _sig(N, 5, "noise"), _sig(N, 6, "noise")
    w = sg.hamming(Np)
    assert np.array_equal(O.ssca_cross(x, x, Np, w), O.ssca(x, Np, w))
    xr = x.real.astype(np.complex128)
    assert np.array_equal(O.ssca_cross(xr, xr, Np, w, conjugate=True), O.ssca(xr, Np, w))
    assert np.abs(O.ssca_cross(x, y, Np, w) - O.ssca_cross(y, x, Np, w)).max() > 1e-3 * np.abs(O.ssca(x, Np, w)).max()


@pytest.mark.parametrize("conjugate", [False, True])
def test_fam_cross_equals_eq5_direct_sum(conjugate):
    """Cross and conjugate FAM cells equal the Eq. (5) sums of Eq. (1) demodulates of x and y (y != x)."""
    Np, L, P = 8, 2, 8
    x, y = _sig(P * L, 7, "noise"), _sig(P * L, 8, "noise")
    w = sg.hamming(Np)
    S = O.fam_cross(x, y, Np, L, P, w, conjugate)
    ref = np.array([[[B.fam_cross_cell_eq15(x, y, list(w), L, P, k, l, q, conjugate) for q in range(P)]
                     for l in range(Np)] for k in range(Np)])
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fam_cross_with_itself_is_the_auto_fam():
    x = _sig(256, 9, "bpsk")
    w = sg.hamming(16)
    assert np.array_equal(O.fam_cross(x, x, 16, 4, 64, w), O.fam(x, 16, 4, 64, w))


def test_ssca_block_pins():
    """The block form over the whole signal is the SSCA; each block cell equals the direct Eq. (1)-(2) sum over
    the block's times with demodulates of the whole signal (edges see the neighbouring samples). The offset is
    a multiple of Np, so the down-conversion of Eq. (3) is the same from the block's start as from the signal's."""
    x = _sig(64, 10, "noise")
    w = sg.hamming(8)
    assert np.array_equal(O.ssca_block(x, 0, 64, 8, w), O.ssca(x, 8, w))
    off, N, Np = 16, 16, 8
    S = O.ssca_block(x, off, N, Np, w)
    d = Np // 2 - 1
    xs, ws = list(x), list(w)
    for k in range(Np):
        for q in range(N):
            acc = 0j
            for n in range(N):
                a = B.demodulate_eq1(xs, off + n, k / Np, ws)
                acc += a * (x[off + n] * np.exp(2j * np.pi * q * n / N)).conjugate()
            ref = np.exp(-2j * np.pi * k * d / Np) * acc
            assert abs(S[k][q] - ref) <= 1e-12 * np.abs(S).max(), (k, q)


def test_ssca_window_orientation_matters():
    """A planted mistake (window reversed, which differs for an asymmetric window) is caught by the Eq. (2) pin."""
    N, Np = 32, 8
    x = _sig(N, 2)
    w = np.linspace(0.1, 1.0, Np)
    S_bad = O.ssca(x, Np, w[::-1])
    ref = np.array([[B.ssca_cell_eq2(list(x), list(w), k, q) for q in range(N)] for k in range(Np)])
    assert np.abs(S_bad - ref).max() > 1e-3 * np.abs(ref).max()
    S_good = O.ssca(x, Np, w)
    assert np.abs(S_good - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("M1", [4, 8, 16])
def test_ssca_2dfft_stage1_stage2_equals_plain(M1):
    """Eq. (10)-(16): the two-stage decomposed DFT with rotation factor, read out at q = m1' + M1*m2'."""
    x = _sig(128, 3)
    w = sg.hamming(16)
    S = O.ssca(x, 16, w)
    S2 = O.ssca_2dfft(x, 16, w, M1)
    assert np.abs(S - S2).max() <= 1e-12 * np.abs(S).max()


def test_ssca_alpha0_is_correlogram_psd():
    """At alpha = 0 (q_c = -k_c N/Np) each strip gives the Blackman-Tukey PSD estimate (alpha = 0 reduces to
    the PSD)."""
    N, Np = 64, 8
    x = _sig(N, 4)
    w = sg.hamming(Np)
    S = O.ssca(x, Np, w)
    for k in range(Np):
        kc = ((k + Np // 2) % Np) - Np // 2
        q = (-kc * N // Np) % N
        ref = B.correlogram_psd(list(x), list(w), k)
        assert abs(S[k, q] - ref) <= 1e-12 * abs(ref)


def test_channelizer_equals_direct_eq3():
    x = _sig(40, 5)
    w = sg.hamming(8)
    XT = O.channelize(x, 8, 2, 20, w)
    ref = np.array(B.channelize_direct(list(x), 8, 2, 20, list(w)))
    assert np.abs(XT - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ssca_fir_channelizer_equals_frame_channelizer():
    """The SSCA's per-channel FIR form and the frame+DFT form of Eq. (3) (L = 1) agree."""
    x = _sig(96, 6)
    w = sg.hamming(16)
    XT = O.channelize(x, 16, 1, 96, w)
    for k in (0, 3, 8, 15):
        assert np.abs(O.ssca_demodulate_strip(x, 16, w, k) - XT[:, k]).max() <= 1e-12 * np.abs(XT).max()


@pytest.mark.parametrize("Np,L,P", [(8, 2, 16), (8, 4, 8)])
def test_fam_equals_eq5_with_eq1_demodulates(Np, L, P):
    x = _sig(P * L + 5, 7)
    w = sg.hamming(Np)
    S = O.fam(x, Np, L, P, w)
    xs, ws = list(x), list(w)
    ref = np.array([[[B.fam_cell_eq15(xs, ws, L, P, k, l, q) for q in range(P)] for l in range(Np)]
                    for k in range(Np)])
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fam_alpha0_is_welch_sum():
    """S[k][k][0] = sum_p |X_T[p][k]|^2, the Welch PSD sum with hop L and window w."""
    Np, L, P = 16, 4, 32
    x = _sig(P * L, 8)
    w = sg.hamming(Np)
    S = O.fam(x, Np, L, P, w)
    XT = np.array(B.channelize_direct(list(x), Np, L, P, list(w)))
    welch = (np.abs(XT) ** 2).sum(axis=0)
    assert np.abs(np.diagonal(S[:, :, 0]) - welch).max() <= 1e-12 * welch.max()


def test_fam_conjugate_symmetry():
    """S[l][k][(-q) mod P] = conj(S[k][l][q])."""
    Np, L, P = 16, 4, 32
    S = O.fam(_sig(P * L, 9), Np, L, P, sg.hamming(Np))
    T = np.conj(S.transpose(1, 0, 2)[:, :, (-np.arange(P)) % P])
    assert np.abs(S - T).max() <= 1e-13 * np.abs(S).max()


def test_scale_and_window_linearity():
    """S(cx) = |c|^2 S(x) for both estimators; SSCA is linear in w and FAM quadratic."""
    x = _sig(256, 10)
    c = 0.3 - 1.7j
    w1, w2 = sg.hamming(16), np.linspace(0.2, 1.0, 16)
    S = O.ssca(x, 16, w1)
    assert np.allclose(O.ssca(c * x, 16, w1), abs(c) ** 2 * S, rtol=0, atol=1e-12 * np.abs(S).max())
    lin = O.ssca(x, 16, 2.0 * w1 - 0.5 * w2)
    assert np.allclose(lin, 2.0 * S - 0.5 * O.ssca(x, 16, w2), rtol=0, atol=1e-12 * np.abs(S).max())
    F = O.fam(x, 16, 4, 64, w1)
    assert np.allclose(O.fam(c * x, 16, 4, 64, w1), abs(c) ** 2 * F, rtol=0, atol=1e-12 * np.abs(F).max())
    assert np.allclose(O.fam(x, 16, 4, 64, 3.0 * w1), 9.0 * F, rtol=0, atol=1e-12 * 9 * np.abs(F).max())


def _alpha_profile(S, a, N):
    ai = np.rint(a * N).astype(np.int64)
    prof = np.zeros(2 * N + 1)
    np.maximum.at(prof, ai.ravel() + N, np.abs(S).ravel())
    return np.arange(-N, N + 1) / N, prof


def test_bpsk_cycle_frequencies():
    """Real-carrier BPSK (fc = 0.05, T_b = 8): the strongest alpha != 0 features sit at +-2fc, +-1/T_b and
    +-(1/T_b -+ 2fc), within one alpha bin."""
    N, Np = 1024, 32
    x = sg.bpsk(N, 0.05, 8, 0.0, sg.rng_for(1, 0))
    S = O.ssca(x, Np, sg.hamming(Np))
    _, a = O.ssca_coords(Np, N)
    al, prof = _alpha_profile(S, a, N)
    prof[np.abs(al) < 4.0 / N] = 0
    top = al[np.argsort(-prof)[:10]]
    expected = np.array([0.1, 0.125, 0.025, 0.225])
    for v in top:
        assert np.min(np.abs(np.abs(v) - expected)) <= 1.0 / N + 1e-12, v
    for e in (0.1, -0.1, 0.125, -0.125):
        assert np.min(np.abs(top - e)) <= 1.0 / N + 1e-12


def test_qpsk_cycle_frequency_symbol_rate():
    """Complex-carrier QPSK with 8 samples/symbol: the strongest alpha != 0 feature is at +-1/8."""
    N, Np = 4096, 32
    x = sg.qpsk(N, 0.1, 8, 5.0, sg.rng_for(91, 0))
    S = O.ssca(x, Np, sg.hamming(Np))
    _, a = O.ssca_coords(Np, N)
    al, prof = _alpha_profile(S, a, N)
    prof[np.abs(al) < 4.0 / N] = 0
    top = al[np.argsort(-prof)[:2]]
    assert np.all(np.abs(np.abs(top) - 0.125) <= 1.0 / N + 1e-12)


def test_ssca_alpha_symmetry_statistical():
    """The alpha-profiles at +alpha and -alpha agree within estimator noise for the BPSK features."""
    N, Np = 1024, 32
    x = sg.bpsk(N, 0.05, 8, 0.0, sg.rng_for(1, 0))
    S = O.ssca(x, Np, sg.hamming(Np))
    _, a = O.ssca_coords(Np, N)
    al, prof = _alpha_profile(S, a, N)
    for e in (0.1, 0.125):
        i_p = np.argmin(np.abs(al - e))
        i_m = np.argmin(np.abs(al + e))
        pp = prof[i_p - 1:i_p + 2].max()
        pm = prof[i_m - 1:i_m + 2].max()
        assert abs(pp - pm) <= 0.1 * max(pp, pm)


def test_dsss_cycle_frequencies_golden():
    """Sec. IV-A: the DSSS BPSK test signal's cycle frequencies are multiples of the data rate 0.25/31."""
    g = json.load(open(os.path.join(GOLDEN, "dsss_bpsk_cycle_frequencies.json")))
    N, Np = 4096, 32
    x = sg.dsss_bpsk(N, g["snr_db"], sg.rng_for(7, 0), chip_rate=g["chip_rate"], gain=g["processing_gain"])
    S = O.ssca(x, Np, sg.hamming(Np))
    _, a = O.ssca_coords(Np, N)
    al, prof = _alpha_profile(S, a, N)
    prof[np.abs(al) < 4.0 / N] = 0
    rate = g["data_rate"]
    assert abs(rate - g["chip_rate"] / g["processing_gain"]) < 1e-15
    for v in al[np.argsort(-prof)[:16]]:
        m = np.rint(v / rate)
        assert m != 0 and abs(v - m * rate) <= 1.0 / N, v


def test_fam_and_ssca_agree_on_strongest_feature():
    """Different estimators of the same SCD: their strongest alpha != 0 features coincide within FAM's
    alpha resolution 1/(P L) (statistical agreement, not equality)."""
    x = sg.bpsk(4096, 0.05, 8, 10.0, sg.rng_for(92, 0))
    N, Np = 4096, 32
    S = O.ssca(x, Np, sg.hamming(Np))
    _, a = O.ssca_coords(Np, N)
    al, prof = _alpha_profile(S, a, N)
    prof[np.abs(al) < 4.0 / N] = 0
    top_ssca = abs(al[np.argmax(prof)])
    Npf, L, P = 32, 8, 512
    F = O.fam(x, Npf, L, P, sg.hamming(Npf))
    _, af = O.fam_coords(Npf, L, P)
    qc = ((np.arange(P) + P // 2) % P) - P // 2
    valid = np.broadcast_to(np.abs(qc) < P // 4, F.shape)
    mag = np.where(valid, np.abs(F), 0.0)
    mag[np.abs(af) < 4.0 / (P * L)] = 0
    top_fam = abs(af.ravel()[np.argmax(mag)])
    assert abs(top_fam - top_ssca) <= 1.0 / (P * L) + 1.0 / N


def test_paper_worked_parameters():
    """Sec. III: the paper's worked FAM and SSCA parameter sets and the SSCA intermediate size."""
    g = json.load(open(os.path.join(GOLDEN, "paper_worked_parameters.json")))
    f = g["fam"]
    assert f["L"] == f["Np"] // 4 and f["P"] == 4 * f["N"] // f["Np"]
    s = g["ssca"]
    assert s["M1"] * s["M2"] == s["N"] and 8 * s["N"] * s["Np"] == s["intermediate_bytes"]
    # The 2-D decomposition at the paper's M1:M2 ratio, scaled down, matches the plain SSCA.
    x = _sig(256, 11)
    w = sg.hamming(16)
    assert np.abs(O.ssca_2dfft(x, 16, w, 16) - O.ssca(x, 16, w)).max() <= 1e-12 * np.abs(O.ssca(x, 16, w)).max()


def test_coordinate_map_matches_brute_force_frequencies():
    """The (f, alpha) assigned to a cell are the f1 = f + alpha/2 = f_k and f2 = f - alpha/2 = -q/N used by
    the Eq. (2) pin (mod 1)."""
    Np, N = 8, 32
    f, a = O.ssca_coords(Np, N)
    for k in range(Np):
        for q in range(N):
            f1 = f[k, q] + a[k, q] / 2
            f2 = f[k, q] - a[k, q] / 2
            assert abs(((f1 - k / Np) + 0.5) % 1.0 - 0.5) < 1e-12
            assert abs(((f2 + q / N) + 0.5) % 1.0 - 0.5) < 1e-12
            assert -0.5 <= f[k, q] <= 0.5 and -1.0 <= a[k, q] <= 1.0


def test_fam_paper_view_is_alg1_write_order():
    """Alg. 1 writes |z_fft|^2 at indices P/2..3P/4-1, then P/4..P/2-1, of the P-point spectrum read in
    centred (fftshifted) order, i.e. q_c = 0..P/4-1 followed by q_c = -P/4..-1. The oracle's view must
    be exactly that, taken here through numpy's fftshift rather than the view's own index list; a view
    shifted by one bin does not match. The kept set is q_c in [-P/4, P/4)."""
    x = _sig(256, 21)
    Np, L, P = 16, 4, 64
    S = O.fam(x, Np, L, P, sg.hamming(Np))
    z_abs = np.abs(np.fft.fftshift(S, axes=-1)) ** 2
    written = np.concatenate([z_abs[..., P // 2:3 * P // 4], z_abs[..., P // 4:P // 2]], axis=-1)
    assert np.array_equal(O.fam_paper_view(S), written)
    shifted = np.abs(S[..., np.r_[1:P // 4 + 1, P - P // 4 + 1:P, 0]]) ** 2
    assert not np.allclose(shifted, written)
    # The kept bins are the ones inside the channel pair's overlap, |alpha - (f_k - f_l)| <= 1/(4L).
    _, a = O.fam_coords(Np, L, P)
    fk = (((np.arange(Np) + Np // 2) % Np) - Np // 2) / Np
    off = a - (fk[:, None] - fk[None, :])[:, :, None]
    kept = np.abs(np.fft.fftshift(off, axes=-1))[..., P // 4:3 * P // 4]
    assert kept.max() <= 1.0 / (4 * L) and np.abs(off).max() > 1.0 / (4 * L)


@pytest.mark.parametrize("ka,kb,qd", [(1, 6, 3), (6, 1, -5), (3, 5, 2), (0, 7, -1)])
def test_fam_coords_place_a_two_tone_cycle_frequency(ka, kb, qd):
    """Two complex tones at f_a = k_a/Np and f_b = k_b/Np + q_d/(P L) have one cycle frequency
    alpha = f_a - f_b (the product x_a conj(x_b)). The Eq. (1)/(5) direct sums of the channel pair (k_a, k_b)
    peak at the bin q whose fam_coords alpha is exactly f_a - f_b (pins the sign of alpha, which operand is
    conjugated, and the spacing 1/(P L)); the cell's f lies within one channel width of (f_a + f_b)/2."""
    Np, L, P = 8, 2, 32
    N = P * L
    n = np.arange(N)
    sgn = lambda k: ((k + Np // 2) % Np) - Np // 2
    fa = sgn(ka) / Np
    fb = sgn(kb) / Np + qd / (P * L)
    x = np.exp(2j * np.pi * fa * n) + np.exp(2j * np.pi * fb * n)
    w = list(sg.hamming(Np))
    row = np.array([B.fam_cell_eq15(x, w, L, P, ka, kb, q) for q in range(P)])
    q = int(np.argmax(np.abs(row)))
    f, a = O.fam_coords(Np, L, P)
    assert abs(a[ka, kb, q] - (fa - fb)) < 1e-12
    assert abs(f[ka, kb, q] - (fa + fb) / 2) <= 1.0 / Np
    # A sign-flipped map (alpha = f_l - f_k - q_c/(P L)) places the same peak at -(f_a - f_b).
    assert abs(-a[ka, kb, q] - (fa - fb)) > 1e-6
