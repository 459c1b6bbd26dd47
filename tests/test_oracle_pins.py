"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it rests on.  None of them retypes the oracle's
formulas: the expected values come from numpy's FFT, SVD, eigh and dense solve,
from closed forms, or from identities between separate oracle calls.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2410_06129_amd import synth


def cartesian_enc(n):
    return synth.Encoding(n, n, synth.cartesian_full(n, n))


def tiny_enc(seed=0, nx=6, ny=5, C=2, K=40, species=None, b0=False):
    rng = np.random.default_rng(seed)
    k = rng.uniform(-max(nx, ny) / 2, max(nx, ny) / 2, size=(K, 2))
    coil = synth.coil_maps(nx, ny, C, rng) if C > 1 else None
    need_t = b0 or (species is not None and len(species) > 1)
    t = synth.sample_times(K, 50e-6) if need_t else None
    b0m = synth.b0_map(nx, ny, rng) if b0 else None
    sp = None if species is None else np.asarray(species, float)
    return synth.Encoding(nx, ny, k, t=t, coil=coil, b0_hz=b0m, species_hz=sp)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- P1: fully sampled Cartesian reduces to the DFT (Sec. 4.2: pinv along a
#         uniformly sampled axis without regularisation equals the 1-D FFT) ---

@pytest.mark.parametrize("n", [4, 8, 10])
def test_p1_cartesian_gram_is_scaled_identity(n):
    enc = cartesian_enc(n)
    G = oracle.gram(enc)
    N = n * n
    assert np.max(np.abs(G - N * np.eye(N))) <= 1e-12 * N


@pytest.mark.parametrize("n", [4, 8])
def test_p1_cartesian_lambda0_is_inverse_dft(n):
    enc = cartesian_enc(n)
    rng = np.random.default_rng(7)
    d = synth.unit_complex_noise((3, n * n), rng)
    x = oracle.reconstruct(enc, d, lam=0.0)
    for f in range(3):
        D = d[f].reshape(n, n)                   # [ky, kx], k = index - n/2
        ref = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(D)))   # [iy, ix]
        assert rel(x[f], ref.ravel()) < 1e-13


def test_p1_cartesian_R_is_scaled_adjoint():
    n, lam = 6, 3.5
    enc = cartesian_enc(n)
    b = oracle.Build(enc, lam=lam)
    R = b.recon_matrix()
    # unitary-up-to-scale E: R = E^H/(N+lam); E^H from numpy's inverse DFT matrix
    N = n * n
    eye = np.eye(N)
    # column j of E^H d for d = e_j is the inverse DFT (times N) of a unit impulse
    cols = []
    for j in range(N):
        D = eye[j].reshape(n, n)
        cols.append(N * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(D))).ravel())
    EH = np.stack(cols, axis=1)
    assert rel(R, EH / (N + lam)) < 1e-13


# --- species and off-resonance factors reduce to a DFT too (Sec. 3.3) ---------

def test_species_factor_is_a_dft_over_time():
    S, dt = 8, 1e-3
    # one voxel, k = 0, species at f_s = s/(S dt), t_i = i dt:  E[i,s] = exp(-i2pi s i/S)
    enc = synth.Encoding(1, 1, np.zeros((S, 2)), t=np.arange(S) * dt,
                         species_hz=np.arange(S) / (S * dt))
    d = synth.unit_complex_noise((2, S), np.random.default_rng(3))
    x = oracle.reconstruct(enc, d, lam=0.0)
    assert rel(x, np.fft.ifft(d, axis=1)) < 1e-13


def test_b0_factor_is_a_dft_over_time():
    V, dt = 8, 1e-3
    enc = synth.Encoding(V, 1, np.zeros((V, 2)), t=np.arange(V) * dt,
                         b0_hz=np.arange(V) / (V * dt))
    d = synth.unit_complex_noise((2, V), np.random.default_rng(4))
    x = oracle.reconstruct(enc, d, lam=0.0)
    assert rel(x, np.fft.ifft(d, axis=1)) < 1e-13


def test_uniform_b0_equals_species_shift():
    """A constant off-resonance b behaves as a single species at b Hz: the two
    factors enter the exponent with the same sign and time axis."""
    base = tiny_enc(seed=5, C=1)
    t = synth.sample_times(base.K, 100e-6)
    e1 = synth.Encoding(base.nx, base.ny, base.k, t=t, b0_hz=np.full(base.V, 37.0))
    e2 = synth.Encoding(base.nx, base.ny, base.k, t=t, species_hz=np.array([37.0]))
    assert np.max(np.abs(oracle.encoding_matrix(e1) - oracle.encoding_matrix(e2))) < 1e-13


def test_cartesian_sign_matches_numpy_forward_fft():
    """data = E x with exp(-i2pi k.r) is numpy's forward FFT up to index shifts."""
    n = 8
    enc = cartesian_enc(n)
    x = synth.unit_complex_noise((1, n * n), np.random.default_rng(8))
    d = oracle.forward(enc, x)[0].reshape(n, n)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x[0].reshape(n, n))))
    assert rel(d, ref) < 1e-13


# --- P2: SVD with Tikhonov filter factors (Eq. 4; Sec. 2.2 eigenvalues = s^2) --

@pytest.mark.parametrize("seed,lam", [(0, 0.3), (1, 5.0), (2, 1e-2)])
def test_p2_matches_svd_filter_factors(seed, lam):
    enc = tiny_enc(seed=seed)
    E = oracle.encoding_matrix(enc)
    U, s, Vh = np.linalg.svd(E, full_matrices=False)
    R_svd = (Vh.conj().T * (s / (s * s + lam))) @ U.conj().T
    R = oracle.Build(enc, lam=lam).recon_matrix()
    kappa = (s[0] ** 2 + lam) / (s[-1] ** 2 + lam)
    assert rel(R, R_svd) < 1e-13 * kappa


# --- P3: Moore-Penrose conditions at lam = 0 (Sec. 2; left pseudoinverse) -----

def test_p3_moore_penrose_conditions():
    enc = tiny_enc(seed=11, K=60)
    E = oracle.encoding_matrix(enc)
    R = oracle.Build(enc, lam=0.0).recon_matrix()
    s = np.linalg.svd(E, compute_uv=False)
    tol = 1e-12 * (s[0] / s[-1]) ** 2
    N = E.shape[1]
    assert rel(E @ R @ E, E) < tol
    assert rel(R @ E @ R, R) < tol
    ER, RE = E @ R, R @ E
    assert np.linalg.norm(ER - ER.conj().T) / np.linalg.norm(ER) < tol
    assert np.linalg.norm(RE - RE.conj().T) / np.linalg.norm(RE) < tol
    assert np.linalg.norm(RE - np.eye(N)) / math.sqrt(N) < tol


# --- P4: large lambda tends to conjugate phase (Sec. 2.2) ---------------------

def test_p4_large_lambda_conjugate_phase():
    enc = tiny_enc(seed=12)
    E = oracle.encoding_matrix(enc)
    gnorm = np.linalg.norm(E, 2) ** 2
    prev = None
    for f in (1e3, 1e5, 1e7):
        lam = f * gnorm
        R = oracle.Build(enc, lam=lam).recon_matrix()
        err = np.linalg.norm(lam * R - E.conj().T) / np.linalg.norm(E.conj().T)
        assert err <= 1.01 * gnorm / lam
        if prev is not None:
            assert err < prev
        prev = err


# --- P5: closed-form diagonal and trace; Hermitian PSD Gram (Sec. 2.2) ---------

@pytest.mark.parametrize("kw", [dict(C=1), dict(C=3), dict(C=2, species=[0.0, 150.0], b0=True)])
def test_p5_closed_form_diagonal(kw):
    enc = tiny_enc(seed=13, **kw)
    G = oracle.gram(enc)
    coilpow = np.ones(enc.V) if enc.coil is None else np.sum(np.abs(enc.coil) ** 2, axis=0)
    want = enc.K * np.tile(coilpow, enc.S)
    assert np.max(np.abs(G.diagonal() - want)) < 1e-12 * np.max(want)
    assert abs(np.trace(G).real - enc.K * enc.S * coilpow.sum()) < 1e-11 * enc.K * enc.S * coilpow.sum()
    assert np.max(np.abs(G - G.conj().T)) < 1e-12 * np.max(want)
    assert np.linalg.eigvalsh(G).min() > -1e-10 * np.max(want)


def test_lambda_definition_on_cartesian():
    """rel * trace(E^H E)/N: with G = N I (fully sampled Cartesian) the shift is rel * N exactly,
    and with C coils of known power it is rel * K * sum_c |C_c|^2 averaged over voxels."""
    n = 6
    b = oracle.Build(cartesian_enc(n), rel=0.25)
    assert b.lam == pytest.approx(0.25 * n * n, rel=1e-14)
    enc = tiny_enc(seed=24, C=3)
    G = oracle.gram(enc)
    want = 1e-3 * enc.K * np.sum(np.abs(enc.coil) ** 2) / enc.V
    assert oracle.lambda_abs(G, 1e-3) == pytest.approx(want, rel=1e-12)


# --- P6: coil-sum identity (Eq. 11) --------------------------------------------

def test_p6_coil_sum_identity():
    enc = tiny_enc(seed=14, C=3)
    G = oracle.gram(enc)
    d = synth.unit_complex_noise((2, enc.M), np.random.default_rng(1))
    b = oracle.adjoint(enc, d)
    Gs = np.zeros_like(G)
    bs = np.zeros_like(b)
    for c in range(enc.C):
        ec = synth.Encoding(enc.nx, enc.ny, enc.k, coil=enc.coil[c:c + 1])
        Gs += oracle.gram(ec)
        bs += oracle.adjoint(ec, d[:, c * enc.K:(c + 1) * enc.K])
    assert rel(Gs, G) < 1e-14
    assert rel(bs, b) < 1e-14


def test_column_accessor_matches_rows():
    enc = tiny_enc(seed=25, C=3, species=[0.0, 90.0], b0=True)
    E = oracle.encoding_matrix(enc)
    cols = [0, 7, 29, 31, 59]
    assert np.max(np.abs(oracle.encoding_columns(enc, cols) - E[:, cols])) < 1e-14
    G = E.conj().T @ E
    a, b = [3, 40, 59], [1, 40, 12]
    assert np.max(np.abs(oracle.gram_entries(enc, a, b, block=17) - G[a, b])) < 1e-12 * np.abs(G).max()


def test_forward_is_adjoint_of_adjoint():
    enc = tiny_enc(seed=15, C=2, species=[0.0, 80.0, 200.0], b0=True)
    rng = np.random.default_rng(2)
    x = synth.unit_complex_noise((1, enc.N), rng)
    d = synth.unit_complex_noise((1, enc.M), rng)
    lhs = np.vdot(d, oracle.forward(enc, x))
    rhs = np.vdot(oracle.adjoint(enc, d), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# --- P7: normal-equation residual (Eq. 6) --------------------------------------

@pytest.mark.parametrize("kw", [dict(C=1), dict(C=3), dict(C=2, species=[0.0, 150.0], b0=True)])
def test_p7_normal_equation_residual(kw):
    enc = tiny_enc(seed=16, K=70, **kw)
    b = oracle.Build(enc, rel=1e-3)
    d = synth.unit_complex_noise((3, enc.M), np.random.default_rng(5))
    x = b.reconstruct(d)
    r = b.normal_residual(d, x)
    ehd = oracle.adjoint(enc, d)
    assert np.max(np.linalg.norm(r, axis=1) / np.linalg.norm(ehd, axis=1)) < 1e-12


# --- P8: push-through identity between over- and underdetermined forms ---------

def test_p8_push_through():
    enc = tiny_enc(seed=17)
    E = oracle.encoding_matrix(enc)
    lam = 0.7
    R = oracle.Build(enc, lam=lam).recon_matrix()
    M = E.shape[0]
    R2 = E.conj().T @ np.linalg.solve(E @ E.conj().T + lam * np.eye(M), np.eye(M))
    assert rel(R, R2) < 1e-12


# --- P8b: the right pseudoinverse for fewer samples than unknowns (Sec. 2.2) ---

def test_p8b_right_pinv_equals_left_with_shift():
    """M < N with lam > 0: E^H (E E^H + lam I)^-1 through the M x M factor equals
    (E^H E + lam I)^-1 E^H through the N x N factor (two independent routes)."""
    enc = tiny_enc(seed=23, C=2, K=9, species=[0.0, 140.0])      # M = 18 < N = 60
    rb = oracle.RightBuild(enc, rel=1e-2)
    lb = oracle.Build(enc, lam=rb.lam)
    assert rb.Gr.shape == (18, 18)
    assert abs(rb.lam - 1e-2 * np.trace(lb.G).real / 60) < 1e-12 * rb.lam
    assert rel(rb.recon_matrix(), lb.recon_matrix()) < 1e-10
    rng = np.random.default_rng(5)
    d = rng.standard_normal((3, 18)) + 1j * rng.standard_normal((3, 18))
    assert rel(rb.reconstruct(d), d @ rb.recon_matrix().T) < 1e-12


def test_p8c_right_pinv_minimum_norm_at_zero_shift():
    """lam = 0, full row rank: R is the Moore-Penrose pseudoinverse (numpy's SVD
    pinv and the four Penrose conditions); R d reproduces the data exactly and
    lies in the range of E^H (the minimum-norm solution)."""
    enc = tiny_enc(seed=24, C=1, K=12)       # M = 12 < N = 30
    E = oracle.encoding_matrix(enc)
    R = oracle.RightBuild(enc, lam=0.0).recon_matrix()
    assert rel(R, np.linalg.pinv(E)) < 1e-9
    assert rel(E @ R @ E, E) < 1e-10
    assert rel(R @ E @ R, R) < 1e-10
    ER, RE = E @ R, R @ E
    assert np.linalg.norm(ER - ER.conj().T) < 1e-10 * np.linalg.norm(ER)
    assert np.linalg.norm(RE - RE.conj().T) < 1e-10 * np.linalg.norm(RE)
    rng = np.random.default_rng(6)
    d = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    x = R @ d
    assert rel(E @ x, d) < 1e-10
    # orthogonal to the null space of E: projection onto range(E^H) keeps x
    Q, _ = np.linalg.qr(E.conj().T)
    assert rel(Q @ (Q.conj().T @ x), x) < 1e-10


# --- P9: decomposition independence: eigen route (Eq. 7) -----------------------

def test_p9_eigen_route():
    enc = tiny_enc(seed=18, C=3)
    E = oracle.encoding_matrix(enc)
    lam = 0.05 * np.trace(E.conj().T @ E).real / E.shape[1]
    G = E.conj().T @ E + lam * np.eye(E.shape[1])
    w, P = np.linalg.eigh(G)
    R_eig = (P / w) @ P.conj().T @ E.conj().T
    R = oracle.Build(enc, lam=lam).recon_matrix()
    assert rel(R, R_eig) < 1e-12


# --- P10: SRF identity (Eq. 9) -------------------------------------------------

def test_p10_srf():
    enc = tiny_enc(seed=19, C=2)
    lam = 0.4
    b = oracle.Build(enc, lam=lam)
    E = oracle.encoding_matrix(enc)
    srf = oracle.srf_matrix(b.recon_matrix(), E)
    Gl = E.conj().T @ E + lam * np.eye(E.shape[1])
    want = np.eye(E.shape[1]) - lam * np.linalg.inv(Gl)
    assert rel(srf, want) < 1e-12
    dg = srf.diagonal()
    assert np.all(dg.real > 0) and np.all(dg.real <= 1 + 1e-12) and np.max(np.abs(dg.imag)) < 1e-12
    n = 4
    cb = oracle.Build(cartesian_enc(n), lam=lam)
    srf_c = oracle.srf_matrix(cb.recon_matrix(), oracle.encoding_matrix(cartesian_enc(n)))
    N = n * n
    assert np.max(np.abs(srf_c - N / (N + lam) * np.eye(N))) < 1e-13


def test_noise_matrix_white_noise():
    """With Psi = I the noise matrix equals G_l^-1 - lam G_l^-2 (Eq. 10)."""
    enc = tiny_enc(seed=20)
    lam = 0.3
    E = oracle.encoding_matrix(enc)
    R = oracle.Build(enc, lam=lam).recon_matrix()
    X = oracle.noise_matrix(R, np.eye(E.shape[0]))
    Gi = np.linalg.inv(E.conj().T @ E + lam * np.eye(E.shape[1]))
    assert rel(X, Gi - lam * Gi @ Gi) < 1e-11


def random_hpd(C, rng):
    a = rng.standard_normal((C, C)) + 1j * rng.standard_normal((C, C))
    return a @ a.conj().T + C * np.eye(C)


def test_noise_matrix_coil_covariance():
    """Coil-correlated noise, Psi = Psi_c (x) I_K (Eq. 10): X equals
    G_l^-1 (E^H Psi E) G_l^-1, with E^H Psi E summed over coil blocks
    sum_{c,c'} Psi_c[c,c'] E_c^H E_c' and the inverse from numpy."""
    enc = tiny_enc(seed=22, C=3, K=30)
    lam = 0.25
    E = oracle.encoding_matrix(enc)
    K, C = enc.K, enc.C
    psi_c = random_hpd(C, np.random.default_rng(7))
    X = oracle.noise_matrix(oracle.Build(enc, lam=lam).recon_matrix(),
                            oracle.coil_noise_covariance(psi_c, K))
    blocks = [E[c * K:(c + 1) * K] for c in range(C)]
    EPE = sum(psi_c[c, c2] * blocks[c].conj().T @ blocks[c2] for c in range(C) for c2 in range(C))
    Gi = np.linalg.inv(E.conj().T @ E + lam * np.eye(E.shape[1]))
    assert rel(X, Gi @ EPE @ Gi) < 1e-11
    d = np.diagonal(X)
    assert np.all(d.real > 0) and np.max(np.abs(d.imag)) < 1e-12 * np.max(d.real)
    # Psi_c = I reduces to the white-noise case
    Xw = oracle.noise_matrix(oracle.Build(enc, lam=lam).recon_matrix(),
                             oracle.coil_noise_covariance(np.eye(C), K))
    assert rel(Xw, Gi - lam * Gi @ Gi) < 1e-11


# --- Cholesky failure and determinism ------------------------------------------

def test_not_pd_without_regularisation_when_underdetermined():
    enc = tiny_enc(seed=21, C=1, K=12)     # M=12 < N=30 -> rank deficient Gram
    with pytest.raises(oracle.NotPositiveDefinite) as ei:
        oracle.Build(enc, lam=0.0)
    assert 12 <= ei.value.column < 30


def test_cholesky_matches_numpy():
    rng = np.random.default_rng(22)
    A = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    H = A @ A.conj().T + 40 * np.eye(40)
    L = oracle.cholesky(H)
    assert rel(L, np.linalg.cholesky(H)) < 1e-14


def test_thread_count_independence():
    threadpoolctl = pytest.importorskip("threadpoolctl")
    enc = tiny_enc(seed=23, nx=12, ny=10, C=3, K=300)
    d = synth.unit_complex_noise((2, enc.M), np.random.default_rng(6))
    with threadpoolctl.threadpool_limits(1):
        x1 = oracle.reconstruct(enc, d, rel=1e-3)
    with threadpoolctl.threadpool_limits(4):
        x4 = oracle.reconstruct(enc, d, rel=1e-3)
    assert rel(x1, x4) < 1e-13


# --- planted mistakes are caught (the mistake is planted in a copy of the oracle
#     on the CPU; the pins above must reject it) ---------------------------------

def test_planted_sign_error_is_caught(monkeypatch):
    import oracle.pinv_oracle as po
    orig = po.encoding_rows

    def flipped(enc, m0, m1):
        return orig(enc, m0, m1).conj()     # exp(+i...) instead of exp(-i...) (coil-free case)
    monkeypatch.setattr(po, "encoding_rows", flipped)
    n = 8
    enc = cartesian_enc(n)
    x = synth.unit_complex_noise((1, n * n), np.random.default_rng(8))
    d = po.forward(enc, x)[0].reshape(n, n)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x[0].reshape(n, n))))
    assert rel(d, ref) > 0.5


def test_planted_transpose_in_cholesky_is_caught(monkeypatch):
    import oracle.pinv_oracle as po
    orig = po.cholesky
    monkeypatch.setattr(po, "cholesky", lambda A: orig(A).conj())
    enc = tiny_enc(seed=0)
    E = po.encoding_matrix(enc)
    U, s, Vh = np.linalg.svd(E, full_matrices=False)
    R_svd = (Vh.conj().T * (s / (s * s + 0.3))) @ U.conj().T
    R = po.Build(enc, lam=0.3).recon_matrix()
    assert rel(R, R_svd) > 1e-6


# --- golden fixture: the oracle's values for two tiny encodings -----------------

def test_oracle_matches_golden_fixture():
    """tests/golden/oracle_tiny.json holds the oracle's Gram, shift, factor, R,
    images and SRF diagonal for two tiny encodings (written by
    tests/golden/make_golden.py, from oracle/ only, to 12 digits).  Recomputing
    them from the stored encodings must agree: a change to the oracle's
    conventions that the other pins miss still shows here."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_tiny.json")
    with open(path) as fh:
        rec = json.load(fh)

    def c(a):
        a = np.asarray(a, dtype=float)
        return a[..., 0] + 1j * a[..., 1]

    for name, case in rec["cases"].items():
        e = case["encoding"]
        enc = synth.Encoding(e["nx"], e["ny"], np.asarray(e["k"]),
                             t=None if e["t"] is None else np.asarray(e["t"]),
                             coil=None if e["coil"] is None else c(e["coil"]),
                             b0_hz=None if e["b0_hz"] is None else np.asarray(e["b0_hz"]),
                             species_hz=None if e["species_hz"] is None else np.asarray(e["species_hz"]))
        v = case["values"]
        b = oracle.Build(enc, rel=1e-2) if enc.M >= enc.N else oracle.RightBuild(enc, rel=1e-2)
        G = b.G if enc.M >= enc.N else b.Gr
        assert abs(b.lam - v["lam"]) <= 1e-12 * v["lam"], name
        R = b.recon_matrix()
        E = oracle.encoding_matrix(enc)
        d = c(v["d"])
        for got, want in ((G, v["G"]), (b.L, v["L"]), (R, v["R"]), (b.reconstruct(d), v["x"]),
                          (np.diagonal(oracle.srf_matrix(R, E)), v["srf_diag"])):
            assert rel(got, c(want)) < 1e-10, name


# --- the error metric: per-frame relative image error (Sec. 3.2 compares images
#     by normalised squared error; the bar is on the largest frame) ------------

def test_relative_error_hand_computed():
    x = np.array([[1 + 1j, 2.0, 0.0], [3.0, 4.0, 0.0], [0.0, 0.0, 0.0]])
    ref = np.array([[1.0, 2.0, 0.0], [0.0, 0.0, 5.0], [1.0, 0.0, 0.0]])
    # frame 0: |x - ref| = |1j| = 1, |ref| = sqrt(5); frame 1: |(3, 4, -5)| = sqrt(50),
    # |ref| = 5; frame 2: |(-1, 0, 0)| = 1, |ref| = 1
    want = np.array([1 / math.sqrt(5), math.sqrt(50) / 5, 1.0])
    got = oracle.relative_error(x, ref)
    assert got.shape == (3,)
    assert np.max(np.abs(got - want)) <= 1e-15
    assert oracle.relative_error(ref, ref).max() == 0.0
    # one frame given as a vector
    assert abs(oracle.relative_error(x[0], ref[0])[0] - 1 / math.sqrt(5)) <= 1e-15


# --- voxel masks (Sec. 3.1 and Sec. 4.4: unknowns restricted to a support) ------

def test_mask_selects_columns_of_the_full_encoding():
    """With a mask the unknowns are the listed voxels: E_mask is the full E
    with the other columns left out, species block by species block."""
    base = tiny_enc(seed=11, nx=7, ny=6, C=3, K=60, species=[0.0, 90.0], b0=True)
    vox = np.array([0, 3, 4, 10, 17, 22, 29, 35, 41], dtype=np.int32)
    masked = synth.Encoding(base.nx, base.ny, base.k, t=base.t, coil=base.coil, b0_hz=base.b0_hz,
                            species_hz=base.species_hz, voxels=vox)
    V = base.nx * base.ny
    cols = np.concatenate([s * V + vox for s in range(base.S)])
    E_full = oracle.encoding_matrix(base)
    E_mask = oracle.encoding_matrix(masked)
    assert masked.N == 2 * len(vox)
    assert np.max(np.abs(E_mask - E_full[:, cols])) == 0.0
    # the column evaluator and the Gram restricted the same way
    assert np.max(np.abs(oracle.encoding_columns(masked, [1, 12]) - E_full[:, cols[[1, 12]]])) == 0.0
    G = oracle.gram(masked)
    assert rel(G, oracle.gram(base)[np.ix_(cols, cols)]) < 1e-14


def test_mask_on_cartesian_is_a_restricted_dft():
    """Fully sampled Cartesian with a circular mask: G = N_grid I on the mask,
    so R = E_mask^H / (N_grid + lam) (Sec. 4.4 masking; P1)."""
    n, lam = 8, 2.5
    vox = synth.circular_mask(n, n)
    enc = synth.Encoding(n, n, synth.cartesian_full(n, n), voxels=vox)
    assert 0 < len(vox) < n * n
    G = oracle.gram(enc)
    assert np.max(np.abs(G - n * n * np.eye(len(vox)))) <= 1e-12 * n * n
    R = oracle.Build(enc, lam=lam).recon_matrix()
    Eh = oracle.encoding_matrix(enc).conj().T
    assert rel(R, Eh / (n * n + lam)) < 1e-13


# --- the Gram's Toeplitz (point-spread) structure: without off-resonance every
#     Fourier factor depends on two voxels through their offset only (Eq. 2,
#     Eq. 11) ---------------------------------------------------------------------

def test_gram_is_psf_of_voxel_offsets():
    """G[a][b] = S[a][b] P(s_a, s_b, ix_b - ix_a, iy_b - iy_a) with S the coil
    cross-products and P a sum over samples of one exponential per offset,
    evaluated here straight from its definition (a DFT of the trajectory on the
    offset grid), not through the oracle's E."""
    enc = tiny_enc(seed=12, nx=6, ny=5, C=2, K=70, species=[0.0, 130.0])
    V, S = enc.V, enc.S
    G = oracle.gram(enc)
    t = enc.t
    f = enc.species_hz
    ix, iy = np.arange(V) % enc.nx, np.arange(V) // enc.nx
    rng = np.random.default_rng(3)
    for _ in range(40):
        a, b = rng.integers(0, S * V, 2)
        sa, va, sb, vb = a // V, a % V, b // V, b % V
        dx, dy = ix[vb] - ix[va], iy[vb] - iy[va]
        P = np.sum(np.exp(-2j * math.pi * (enc.k[:, 0] * dx / enc.nx + enc.k[:, 1] * dy / enc.ny
                                           + (f[sb] - f[sa]) * t)))
        Sab = np.sum(enc.coil[:, va].conj() * enc.coil[:, vb])
        assert abs(G[a, b] - Sab * P) <= 1e-12 * abs(G).max()


# --- the eigenvalue route with truncation (Eq. 7; truncated SVD, Eq. 4) ---------

def test_kept_count_hand_computed():
    mu = np.array([16.0, 9.0, 4.0, 1.0, 0.25])          # sigma = 4, 3, 2, 1, 0.5
    assert oracle.kept_count(mu, "none") == 5
    # condition number of the kept set: sigma_1 / sigma_j <= kappa
    assert oracle.kept_count(mu, "kappa", 2.0) == 3       # 4/2 = 2 kept, 4/1 = 4 not
    assert oracle.kept_count(mu, "kappa", 3.99) == 3
    assert oracle.kept_count(mu, "kappa", 4.0) == 4
    assert oracle.kept_count(mu, "kappa", 1.0) == 1
    # energy: sum mu = 30.25; 16 + 9 = 25 (82.6%), + 4 = 29 (95.9%), + 1 = 30 (99.2%)
    assert oracle.kept_count(mu, "energy", 0.80) == 2
    assert oracle.kept_count(mu, "energy", 25.0 / 30.25) == 2
    assert oracle.kept_count(mu, "energy", 0.95) == 3
    assert oracle.kept_count(mu, "energy", 0.99) == 4
    assert oracle.kept_count(mu, "energy", 1.0) == 5


@pytest.mark.parametrize("mode,value", [("kappa", 20.0), ("energy", 0.95), ("none", None)])
def test_eigen_route_truncation_equals_truncated_svd(mode, value):
    """Eq. 4: truncating the SVD of E keeps the same singular vectors the
    Gram's eigendecomposition gives (mu = sigma^2), so with lam = 0,
    P_r diag(1/mu) P_r^H E^H = V_r Sigma_r^-1 U_r^H, computed here from
    numpy's SVD of the explicit E, a route that never forms E^H E."""
    enc = tiny_enc(seed=21, nx=6, ny=5, C=3, K=50)
    E = oracle.encoding_matrix(enc)
    U, sv, Vh = np.linalg.svd(E, full_matrices=False)
    if mode == "kappa":
        r = int(np.sum(sv[0] / sv <= value))
    elif mode == "energy":
        c = np.cumsum(sv ** 2)
        r = int(np.argmax(c >= value * c[-1]) + 1)
    else:
        r = len(sv)
    assert 1 < r <= len(sv)
    R_svd = (Vh[:r].conj().T / sv[:r]) @ U[:, :r].conj().T
    b = oracle.EigenBuild(enc, lam=0.0, mode=mode, value=value)
    assert b.rank == r
    assert np.allclose(b.mu, sv ** 2, rtol=1e-10, atol=1e-10 * sv[0] ** 2)
    kappa = sv[0] / sv[r - 1]
    assert rel(b.recon_matrix(), R_svd) < 1e-12 * kappa ** 2
    d = synth.unit_complex_noise((2, enc.M), np.random.default_rng(4))
    assert rel(b.reconstruct(d), d @ R_svd.T) < 1e-12 * kappa ** 2


def test_eigen_route_without_truncation_equals_cholesky():
    """Eq. 7 with only the shift: the same R as the Cholesky route (Eq. 8)."""
    enc = tiny_enc(seed=22, nx=5, ny=6, C=2, K=60, species=[0.0, 80.0], b0=True)
    e = oracle.EigenBuild(enc, rel=1e-2)
    c = oracle.Build(enc, rel=1e-2)
    assert e.lam == c.lam and e.rank == enc.N
    assert rel(e.recon_matrix(), c.recon_matrix()) < 1e-11


def test_eigen_route_cartesian_closed_form():
    """Fully sampled Cartesian: every eigenvalue of E^H E is N, so any kappa
    keeps them all and R = E^H / (N + lam) (P1)."""
    n, lam = 6, 1.5
    enc = cartesian_enc(n)
    b = oracle.EigenBuild(enc, lam=lam, mode="kappa", value=1.0 + 1e-9)
    assert b.rank == n * n
    assert np.max(np.abs(b.mu - n * n)) < 1e-12 * n * n
    Eh = oracle.encoding_matrix(enc).conj().T
    assert rel(b.recon_matrix(), Eh / (n * n + lam)) < 1e-13
