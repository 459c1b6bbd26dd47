"""FP64 CPU oracle for Pinv-Recon's Cholesky route.  TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this module.  The device library never calls it and shares no code
with it.  It is slow on purpose: every step is the plain definition, in
complex128, so it can be checked against the paper by eye.

What it computes (paper Sec. 2.2, Eq. 6 and Eq. 8):

    G   = E^H E                      (Gram matrix, Hermitian PSD)
    G_l = G + lam * I                (Tikhonov shift; `lam` is the paper's lambda^2)
    G_l = L L^H                      (Cholesky, L lower triangular)
    x   = L^-H L^-1 E^H d            (regularised least-squares image)
    R   = L^-H L^-1 E^H              (the reconstruction matrix, formed for small N)

and, for fewer samples than unknowns, the right pseudoinverse (Sec. 2.2)

    R   = E^H (E E^H + lam I)^-1     (RightBuild; minimum-norm solution at lam = 0)

and the eigenvalue route with truncation (Eq. 7, Eq. 4)

    E^H E = P Lambda P^H,  R = P_r diag(1/(mu_j + lam)) P_r^H E^H  (EigenBuild)

where P_r holds the eigenvectors of the r eigenvalues a truncation keeps.

The encoding element (paper Eq. 2 and the generalised product form of Sec. 3.3,
with the sign convention exp(-i 2 pi ...) used throughout this project):

    E[(c,i),(s,v)] = C_c(v) * exp(-i 2 pi (k_i . r_v + (f_s + B0(v)) t_i))

Rows m = c*K + i (coil-major), columns n = s*V + v with v = iy*nx + ix, or,
when a voxel mask restricts the unknowns to a region (Sec. 3.1, Sec. 4.4),
v = the position in the mask's ascending list of grid indices.
Voxel centres r_v = ((ix - nx/2)/nx, (iy - ny/2)/ny) in FOV units, k in
cycles/FOV, frequencies in Hz, times in seconds.

Each function names the passage it follows.  Pins for every step live in
tests/test_oracle_pins.py (Cartesian inverse DFT, DFT special cases for the
species and off-resonance factors, SVD filter factors, Moore-Penrose
conditions, conjugate-phase limit, closed-form diagonal, coil-sum identity,
normal-equation residual, push-through identity, eigen route, SRF identity,
noise matrix for white and coil-correlated noise, the truncated eigenvalue
route against numpy's SVD of E, voxel masks, the Gram's offset structure).
"""
from __future__ import annotations

import math

import numpy as np

ROW_BLOCK = 4096


class NotPositiveDefinite(ArithmeticError):
    """Raised by `cholesky` when a pivot is not > 0; `.column` names it."""

    def __init__(self, column: int, pivot: float):
        super().__init__(f"matrix is not positive definite: pivot {pivot!r} at column {column}")
        self.column = column
        self.pivot = pivot


# ----------------------------------------------------------------------------
# the encoding matrix  (Eq. 1, Eq. 2; generalised product encoding, Sec. 3.3)
# ----------------------------------------------------------------------------

def unknown_voxels(enc) -> np.ndarray:
    """Grid indices v = iy*nx + ix of the unknowns: every voxel, or the listed
    ones when a mask restricts the unknowns to a region (Sec. 3.1, Sec. 4.4)."""
    if getattr(enc, "voxels", None) is None:
        return np.arange(enc.nx * enc.ny)
    return np.asarray(enc.voxels, dtype=np.int64)


def _dims(enc):
    V = len(unknown_voxels(enc))
    S = 1 if enc.species_hz is None else len(enc.species_hz)
    K = enc.k.shape[0]
    C = 1 if enc.coil is None else enc.coil.shape[0]
    return V, S, K, C


def voxel_positions(nx: int, ny: int):
    x = (np.arange(nx, dtype=np.float64) - nx / 2.0) / nx
    y = (np.arange(ny, dtype=np.float64) - ny / 2.0) / ny
    X, Y = np.meshgrid(x, y)
    return X.ravel(), Y.ravel()


def _unknown_positions(enc):
    """Centres, off-resonance and coil maps at the unknown voxels."""
    g = unknown_voxels(enc)
    X, Y = voxel_positions(enc.nx, enc.ny)
    b0 = np.zeros(len(g)) if enc.b0_hz is None else np.asarray(enc.b0_hz, float)[g]
    coil = None if enc.coil is None else enc.coil[:, g]
    return X[g], Y[g], b0, coil


def encoding_rows(enc, m0: int, m1: int) -> np.ndarray:
    """Rows m0..m1-1 of E, explicitly, [m1-m0, N] complex128.

    Phase in turns = k.r + (f_s + B0) t, reduced to (-1/2, 1/2] before the
    trigonometric functions so the FP64 angle keeps full relative accuracy.
    """
    V, S, K, C = _dims(enc)
    X, Y, b0, coil = _unknown_positions(enc)
    m = np.arange(m0, m1)
    c = m // K
    i = m % K
    kx = enc.k[i, 0][:, None]
    ky = enc.k[i, 1][:, None]
    spatial = kx * X[None, :] + ky * Y[None, :]                    # [rows, V]
    species = np.zeros(S) if enc.species_hz is None else np.asarray(enc.species_hz, float)
    t = np.zeros(K) if enc.t is None else np.asarray(enc.t, float)
    blocks = []
    for s in range(S):
        turns = spatial + (species[s] + b0[None, :]) * t[i][:, None]
        frac = turns - np.round(turns)
        phase = np.cos(2.0 * math.pi * frac) - 1j * np.sin(2.0 * math.pi * frac)
        if coil is not None:
            phase = phase * coil[c, :]
        blocks.append(phase)
    return np.concatenate(blocks, axis=1)


def encoding_columns(enc, cols, m0: int = 0, m1: int = None) -> np.ndarray:
    """Columns `cols` of E over rows m0..m1-1 (all rows by default), [rows, len(cols)];
    the same element definition as encoding_rows, evaluated for chosen columns."""
    V, S, K, C = _dims(enc)
    m1 = C * K if m1 is None else m1
    cols = np.asarray(cols)
    s_idx = cols // V
    v_idx = cols % V
    X, Y, b0, coil = _unknown_positions(enc)
    m = np.arange(m0, m1)
    c = m // K
    i = m % K
    species = np.zeros(S) if enc.species_hz is None else np.asarray(enc.species_hz, float)
    t = np.zeros(K) if enc.t is None else np.asarray(enc.t, float)
    turns = (enc.k[i, 0][:, None] * X[v_idx][None, :] + enc.k[i, 1][:, None] * Y[v_idx][None, :]
             + (species[s_idx][None, :] + b0[v_idx][None, :]) * t[i][:, None])
    frac = turns - np.round(turns)
    out = np.cos(2.0 * math.pi * frac) - 1j * np.sin(2.0 * math.pi * frac)
    if coil is not None:
        out = out * coil[c[:, None], v_idx[None, :]]
    return out


def gram_entries(enc, a, b, block: int = 65536) -> np.ndarray:
    """G[a_j, b_j] = sum_m conj(E[m, a_j]) E[m, b_j] for index pairs (a_j, b_j)."""
    V, S, K, C = _dims(enc)
    a = np.asarray(a)
    b = np.asarray(b)
    out = np.zeros(len(a), dtype=np.complex128)
    for m0 in range(0, C * K, block):
        m1 = min(C * K, m0 + block)
        out += np.sum(encoding_columns(enc, a, m0, m1).conj() * encoding_columns(enc, b, m0, m1), axis=0)
    return out


def encoding_matrix(enc) -> np.ndarray:
    """The whole E, [M, N] (small cases only)."""
    V, S, K, C = _dims(enc)
    return encoding_rows(enc, 0, C * K)


def _row_blocks(enc):
    """Row ranges coil by coil (Eq. 11), each split into <= ROW_BLOCK rows."""
    V, S, K, C = _dims(enc)
    for c in range(C):
        for i0 in range(0, K, ROW_BLOCK):
            yield c * K + i0, c * K + min(K, i0 + ROW_BLOCK)


# ----------------------------------------------------------------------------
# Gram matrix and regularisation  (Sec. 2.2; Eq. 6; Eq. 11)
# ----------------------------------------------------------------------------

def gram(enc) -> np.ndarray:
    """G = E^H E accumulated as the sum of per-coil products E_c^H E_c (Eq. 11)."""
    V, S, K, C = _dims(enc)
    N = S * V
    G = np.zeros((N, N), dtype=np.complex128)
    for m0, m1 in _row_blocks(enc):
        Eb = encoding_rows(enc, m0, m1)
        G += Eb.conj().T @ Eb
    return G


def adjoint(enc, d: np.ndarray) -> np.ndarray:
    """E^H d for frames d [F, M] -> [F, N], summed coil by coil (Eq. 11 remark)."""
    d = np.atleast_2d(d)
    V, S, K, C = _dims(enc)
    out = np.zeros((d.shape[0], S * V), dtype=np.complex128)
    for m0, m1 in _row_blocks(enc):
        Eb = encoding_rows(enc, m0, m1)
        out += d[:, m0:m1] @ Eb.conj()
    return out


def forward(enc, x: np.ndarray) -> np.ndarray:
    """data = E x (Eq. 1) for images x [F, N] -> [F, M]."""
    x = np.atleast_2d(x)
    V, S, K, C = _dims(enc)
    out = np.empty((x.shape[0], C * K), dtype=np.complex128)
    for m0, m1 in _row_blocks(enc):
        Eb = encoding_rows(enc, m0, m1)
        out[:, m0:m1] = x @ Eb.T
    return out


def lambda_abs(G: np.ndarray, rel: float) -> float:
    """Diagonal shift rel * trace(E^H E) / N (= rel * mean diagonal)."""
    return float(rel * np.trace(G).real / G.shape[0])


# ----------------------------------------------------------------------------
# Cholesky and triangular solves  (Eq. 8)
# ----------------------------------------------------------------------------

def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower L with A = L L^H, column by column (Cholesky-Crout), no pivoting.

    L[j,j] = sqrt(A[j,j] - sum_k |L[j,k]|^2)
    L[i,j] = (A[i,j] - sum_k L[i,k] conj(L[j,k])) / L[j,j],  i > j
    Raises NotPositiveDefinite if a pivot is not > 0 (or is NaN).
    """
    N = A.shape[0]
    L = np.zeros_like(A, dtype=np.complex128)
    for j in range(N):
        lj = L[j, :j]
        piv = A[j, j].real - float(np.vdot(lj, lj).real)
        if not piv > 0.0:
            raise NotPositiveDefinite(j, piv)
        ljj = math.sqrt(piv)
        L[j, j] = ljj
        if j + 1 < N:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ lj.conj()) / ljj
    return L


def forward_substitution(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve L Y = B (B is [N, ncols]) row by row."""
    N = L.shape[0]
    Y = np.zeros_like(B, dtype=np.complex128)
    for i in range(N):
        Y[i] = (B[i] - L[i, :i] @ Y[:i]) / L[i, i]
    return Y


def back_substitution_h(L: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Solve L^H X = Y (L lower, so L^H upper) from the last row up."""
    N = L.shape[0]
    X = np.zeros_like(Y, dtype=np.complex128)
    for i in range(N - 1, -1, -1):
        # (L^H)[i, j] = conj(L[j, i]) for j > i
        X[i] = (Y[i] - L[i + 1:, i].conj() @ X[i + 1:]) / np.conj(L[i, i])
    return X


def solve_normal(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X = (L L^H)^-1 B = L^-H L^-1 B."""
    return back_substitution_h(L, forward_substitution(L, B))


# ----------------------------------------------------------------------------
# the method end to end  (Eq. 3, Eq. 6, Eq. 8)
# ----------------------------------------------------------------------------

class Build:
    """The data-independent part: Gram, shift and factor (computed once, reused
    for every frame of every acquisition with the same encoding)."""

    def __init__(self, enc, rel: float = None, lam: float = None, G: np.ndarray = None):
        self.enc = enc
        self.G = gram(enc) if G is None else G
        if (rel is None) == (lam is None):
            raise ValueError("give exactly one of rel or lam")
        self.lam = lambda_abs(self.G, rel) if lam is None else float(lam)
        N = self.G.shape[0]
        self.L = cholesky(self.G + self.lam * np.eye(N))

    def reconstruct(self, d: np.ndarray) -> np.ndarray:
        """Images x = (E^H E + lam I)^-1 E^H d for frames d [F, M] -> [F, N]."""
        b = adjoint(self.enc, d)                 # [F, N]
        return solve_normal(self.L, b.T).T

    def recon_matrix(self) -> np.ndarray:
        """R = L^-H L^-1 E^H, [N, M] (small N only)."""
        Eh = encoding_matrix(self.enc).conj().T
        return solve_normal(self.L, Eh)

    def normal_residual(self, d: np.ndarray, x: np.ndarray) -> np.ndarray:
        """E^H (d - E x) - lam x, per frame [F, N] (zero at the exact solution)."""
        return adjoint(self.enc, np.atleast_2d(d) - forward(self.enc, x)) - self.lam * np.atleast_2d(x)


def reconstruct(enc, d: np.ndarray, rel: float = None, lam: float = None) -> np.ndarray:
    return Build(enc, rel=rel, lam=lam).reconstruct(d)


# ----------------------------------------------------------------------------
# underdetermined problems: the right pseudoinverse  (Sec. 2.2)
# ----------------------------------------------------------------------------

def gram_rows(enc) -> np.ndarray:
    """G' = E E^H, [M, M]: the samples' Gram matrix (small M only)."""
    E = encoding_matrix(enc)
    return E @ E.conj().T


class RightBuild:
    """Fewer samples than unknowns (M < N): R = E^H (E E^H + lam I)^-1, the
    minimum-norm solution for lam = 0 (Sec. 2.2), through the Cholesky factor
    of the M x M matrix E E^H + lam I = L' L'^H.  The shift is given in
    absolute terms or as rel * trace(E E^H) / N, the same trace as E^H E's, so
    for lam > 0 this R equals Build's (push-through identity)."""

    def __init__(self, enc, rel: float = None, lam: float = None):
        self.enc = enc
        self.Gr = gram_rows(enc)
        if (rel is None) == (lam is None):
            raise ValueError("give exactly one of rel or lam")
        N = _dims(enc)[0] * _dims(enc)[1]
        self.lam = float(rel * np.trace(self.Gr).real / N) if lam is None else float(lam)
        M = self.Gr.shape[0]
        self.L = cholesky(self.Gr + self.lam * np.eye(M))

    def recon_matrix(self) -> np.ndarray:
        """R = E^H L'^-H L'^-1 = (L'^-H L'^-1 E)^H, [N, M]."""
        return solve_normal(self.L, encoding_matrix(self.enc)).conj().T

    def reconstruct(self, d: np.ndarray) -> np.ndarray:
        """Images x = E^H (E E^H + lam I)^-1 d for frames d [F, M] -> [F, N]."""
        y = solve_normal(self.L, np.atleast_2d(d).T)   # [M, F]
        return adjoint(self.enc, y.T)


# ----------------------------------------------------------------------------
# the eigenvalue route with truncation  (Eq. 7; truncated SVD, Eq. 4)
# ----------------------------------------------------------------------------

def kept_count(mu: np.ndarray, mode: str, value: float = None) -> int:
    """How many of the eigenvalues mu of E^H E, sorted descending, a truncation
    keeps (Sec. 2.1, Sec. 2.2):
      'none'    all of them;
      'kappa'   those whose singular value sigma_j = sqrt(mu_j) is within a
                condition number `value` of the largest: sigma_1 / sigma_j <= value;
      'energy'  the fewest largest ones whose sum reaches the fraction `value`
                of the total sum (the energy of E, sum of sigma_j^2)."""
    mu = np.asarray(mu, dtype=np.float64)
    if mode == "none":
        return len(mu)
    if mode == "kappa":
        return int(np.sum(mu * value * value >= mu[0]))
    if mode == "energy":
        c = np.cumsum(mu)
        return int(np.searchsorted(c, value * c[-1], side="left") + 1)
    raise ValueError(mode)


class EigenBuild:
    """Eq. 7: the Gram's eigendecomposition E^H E = P Lambda P^H (library eigh,
    FP64), then R = P_r diag(f) P_r^H E^H over the r eigenvalues the
    truncation keeps (largest first), with f_j = 1 / (mu_j + lam): truncation
    alone (lam = 0) is the truncated SVD of Eq. 4, the shift alone is Tikhonov
    regularisation, and both can be combined."""

    def __init__(self, enc, lam: float = 0.0, rel: float = None, mode: str = "none",
                 value: float = None, G: np.ndarray = None):
        self.enc = enc
        self.G = gram(enc) if G is None else G
        self.lam = lambda_abs(self.G, rel) if rel is not None else float(lam)
        mu, P = np.linalg.eigh(self.G)
        order = np.argsort(-mu, kind="stable")
        self.mu = mu[order]
        self.P = P[:, order]
        self.rank = kept_count(self.mu, mode, value)
        self.f = 1.0 / (self.mu[:self.rank] + self.lam)

    def recon_matrix(self) -> np.ndarray:
        Pr = self.P[:, :self.rank]
        Eh = encoding_matrix(self.enc).conj().T
        return (Pr * self.f) @ (Pr.conj().T @ Eh)

    def reconstruct(self, d: np.ndarray) -> np.ndarray:
        Pr = self.P[:, :self.rank]
        b = adjoint(self.enc, d)                  # [F, N]
        return ((b @ Pr.conj()) * self.f) @ Pr.T


# ----------------------------------------------------------------------------
# image metrics from R  (Eq. 9, Eq. 10)
# ----------------------------------------------------------------------------

def srf_matrix(R: np.ndarray, E: np.ndarray) -> np.ndarray:
    """SRF = R E (Eq. 9); its diagonal reshaped to the grid is the SRF map."""
    return R @ E


def noise_matrix(R: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """X = R Psi R^H for a data-noise covariance Psi [M, M] (Eq. 10)."""
    return R @ psi @ R.conj().T


def coil_noise_covariance(psi_c: np.ndarray, K: int) -> np.ndarray:
    """Data-noise covariance [M, M] for noise that is white over the K samples
    and correlated over coils with covariance psi_c [C, C]: entry
    ((c, i), (c', i')) is psi_c[c, c'] when i == i', else 0, with rows in the
    coil-major order m = c*K + i of E.  This is the Psi of Eq. 10."""
    psi_c = np.asarray(psi_c, dtype=np.complex128)
    C = psi_c.shape[0]
    psi = np.zeros((C * K, C * K), dtype=np.complex128)
    for c in range(C):
        for c2 in range(C):
            psi[c * K:(c + 1) * K, c2 * K:(c2 + 1) * K] = psi_c[c, c2] * np.eye(K)
    return psi


def relative_error(x: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-frame ||x - ref|| / ||ref|| for [F, N] arrays."""
    x = np.atleast_2d(x)
    ref = np.atleast_2d(ref)
    return np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)
