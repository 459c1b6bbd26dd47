"""The eigenvalue route (Eq. 7) with truncation (Sec. 2.1, Eq. 4) on the HIP
path (Jacobi eigendecomposition of the FP64 Gram, then W = Q^H E^H and R = Q W
with Q = P_r diag(1/sqrt(mu_j + lam))), against the oracle's EigenBuild
(numpy's eigh of the FP64 Gram; pinned against the SVD of E).

* Eigenvalues: within 1e-12 of the largest (Jacobi and eigh are both
  backward stable: errors of order N u ||G||).
* Truncation thresholds are placed in the middle of the widest gap of the
  oracle's spectrum, so no eigenvalue sits within rounding of the threshold;
  the kept count must equal the oracle's.
* FP64 plans: R element by element within 1e-8 of max|R| (the kept
  eigenvectors' error, u ||G|| / gap, amplified by the kept condition number
  mu_1 / mu_r, which the choice of cut keeps within 1e4); images within 1e-8.
* FP32 plans: images within (mu_1 + lam) / (mu_r + lam) * 1e-6.
* Odd N (the Jacobi ordering pads one index), a voxel mask and N = 1024 (about
  30 sweeps) are covered.
"""
import numpy as np
import pytest

import oracle
from paper_2410_06129_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    from paper_2410_06129_amd import pinv
    return pinv


@pytest.fixture(scope="module")
def ctx(P):
    assert torch.cuda.is_available()
    c = P.pinv_context_create(0)
    yield c
    P.pinv_context_destroy(c)


def encoding(name):
    if name == "even_c3":      # N = 480
        return synth.small_case(seed=501, nx=24, ny=20, C=3, K=700, F=1).enc
    if name == "odd_species":   # two species on a 13 x 11 grid (N = 286), MFMA Gram
        return synth.small_case(seed=502, nx=13, ny=11, C=2, K=600, F=1, species=[0.0, 170.0],
                                b0=True).enc
    if name == "odd_c2":        # N = 13 * 11 = 143, odd
        return synth.small_case(seed=503, nx=13, ny=11, C=2, K=400, F=1).enc
    if name == "n1024":         # 32 x 32, 8 coils, spiral of 2N per coil (M = 16384)
        return synth.serving_encoding(32, 8, 0)
    if name == "masked":        # circular mask, N odd or even as it falls
        w = synth.small_case(seed=504, nx=22, ny=22, C=2, K=900, F=1)
        e = w.enc
        return synth.Encoding(e.nx, e.ny, e.k, coil=e.coil, voxels=synth.circular_mask(22, 22))
    raise KeyError(name)


_cache = {}


def oracle_spectrum(name):
    if name not in _cache:
        enc = encoding(name)
        G = oracle.gram(enc)
        base = oracle.EigenBuild(enc, lam=0.0, G=G)
        _cache[name] = (enc, G, base.mu)
    return _cache[name]


def gap_kappa(mu, lo=0.2, hi=0.7, max_cond=1e4):
    """A condition number whose threshold mu_0 / kappa^2 lies in the middle (on a
    log scale) of the widest relative gap between eigenvalues ranked lo..hi,
    among cuts whose kept condition mu_0 / mu_r stays within max_cond (the
    tolerances below assume it; the species case reaches 9e9 at rank 200)."""
    n = len(mu)
    js = [j for j in range(int(lo * n), int(hi * n)) if mu[0] <= max_cond * mu[j]]
    j = max(js, key=lambda j: mu[j] / mu[j + 1])
    thr = np.sqrt(mu[j] * mu[j + 1])
    return float(np.sqrt(mu[0] / thr)), j + 1


def gap_energy(mu, lo=0.2, hi=0.7):
    """An energy fraction half-way between the running sums of two neighbours
    around the widest gap (so the kept count is j + 1)."""
    c = np.cumsum(mu)
    _, r = gap_kappa(mu, lo, hi)
    return float((c[r - 2] + c[r - 1]) / 2 / c[-1]), r


def run(P, ctx, enc, prec, lam, mode, trunc, value, F=3, seed=9):
    N, M = enc.N, enc.M
    cdt = np.complex128 if prec == P.FP64 else np.complex64
    plan = P.pinv_build(ctx, enc, lam, mode, prec, P.FLAG_UNCACHED, route=P.ROUTE_EIGEN,
                        trunc=trunc, trunc_value=value)
    try:
        P.pinv_plan_wait(plan)
        info = P.pinv_plan_info_get(plan)
        spec = torch.empty((N,), dtype=torch.float64, device="cuda")
        P.pinv_spectrum(ctx, plan, spec)
        R = torch.empty((N, M), dtype=torch.complex128 if prec == P.FP64 else torch.complex64,
                        device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        rng = np.random.default_rng(seed)
        d = synth.random_frames((F, M), rng)
        x = torch.empty((F, N), dtype=R.dtype, device="cuda")
        P.pinv_apply(ctx, plan, torch.from_numpy(d.astype(cdt)).cuda(), x)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    return info, spec.cpu().numpy(), R.cpu().numpy().astype(np.complex128), d, \
        x.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("name", ["even_c3", "odd_c2", "odd_species", "masked"])
@pytest.mark.parametrize("how", ["tikhonov", "kappa", "energy", "kappa+shift"])
def test_eigen_route_fp64_matches_oracle(P, ctx, name, how):
    enc, G, mu = oracle_spectrum(name)
    lam_abs = 1e-3 * np.trace(G).real / enc.N
    if how == "tikhonov":
        trunc, value, lam = P.TRUNC_NONE, 0.0, lam_abs
    elif how == "kappa":
        (value, _), trunc, lam = gap_kappa(mu), P.TRUNC_KAPPA, 0.0
    elif how == "energy":
        (value, _), trunc, lam = gap_energy(mu), P.TRUNC_ENERGY, 0.0
    else:
        (value, _), trunc, lam = gap_kappa(mu), P.TRUNC_KAPPA, lam_abs
    mode = {P.TRUNC_NONE: "none", P.TRUNC_KAPPA: "kappa", P.TRUNC_ENERGY: "energy"}[trunc]
    ob = oracle.EigenBuild(enc, lam=lam, mode=mode, value=value, G=G)
    info, spec, R, d, x = run(P, ctx, enc, P.FP64, lam, P.LAMBDA_ABS, trunc, value)
    print(f"{name} {how}: rank {info['rank']} / {enc.N} (oracle {ob.rank}), {info['sweeps']} sweeps")
    assert info["route"] == P.ROUTE_EIGEN and info["sweeps"] > 0
    assert info["rank"] == ob.rank
    assert np.max(np.abs(spec - ob.mu)) <= 1e-12 * ob.mu[0]
    R_ref = ob.recon_matrix()
    assert np.max(np.abs(R - R_ref)) <= 1e-8 * np.max(np.abs(R_ref))
    xr = ob.reconstruct(d)
    assert np.max(np.linalg.norm(x - xr, axis=1) / np.linalg.norm(xr, axis=1)) < 1e-8


def test_eigen_route_at_n1024_matches_oracle(P, ctx):
    """N = 1024, where the Jacobi solver needs about 30 sweeps (ill-conditioned
    Gram, clustered small eigenvalues): spectrum, kept rank, R and images of a
    kappa-truncated FP64 plan against the oracle, at the bars above."""
    enc, G, mu = oracle_spectrum("n1024")
    value, r = gap_kappa(mu)
    ob = oracle.EigenBuild(enc, lam=0.0, mode="kappa", value=value, G=G)
    assert ob.rank == r
    info, spec, R, d, x = run(P, ctx, enc, P.FP64, 0.0, P.LAMBDA_ABS, P.TRUNC_KAPPA, value)
    print(f"n1024: rank {info['rank']} / {enc.N}, {info['sweeps']} sweeps")
    assert info["sweeps"] > 0 and info["rank"] == ob.rank
    assert np.max(np.abs(spec - ob.mu)) <= 1e-12 * ob.mu[0]
    R_ref = ob.recon_matrix()
    assert np.max(np.abs(R - R_ref)) <= 1e-8 * np.max(np.abs(R_ref))
    xr = ob.reconstruct(d)
    assert np.max(np.linalg.norm(x - xr, axis=1) / np.linalg.norm(xr, axis=1)) < 1e-8


@pytest.mark.parametrize("how", ["tikhonov", "kappa"])
def test_eigen_route_fp32(P, ctx, how):
    enc, G, mu = oracle_spectrum("even_c3")
    lam_abs = 1e-3 * np.trace(G).real / enc.N
    if how == "tikhonov":
        trunc, value, lam, mode = P.TRUNC_NONE, 0.0, lam_abs, "none"
    else:
        (value, _), trunc, lam, mode = gap_kappa(mu), P.TRUNC_KAPPA, 0.0, "kappa"
    ob = oracle.EigenBuild(enc, lam=lam, mode=mode, value=value, G=G)
    info, spec, R, d, x = run(P, ctx, enc, P.FP32, lam, P.LAMBDA_ABS, trunc, value)
    assert info["rank"] == ob.rank
    cond = (ob.mu[0] + lam) / (ob.mu[ob.rank - 1] + lam)
    xr = ob.reconstruct(d)
    err = np.max(np.linalg.norm(x - xr, axis=1) / np.linalg.norm(xr, axis=1))
    print(f"fp32 {how}: rank {info['rank']}, kept condition {cond:.3g}, error {err:.2e}")
    assert err < cond * 1e-6


def test_eigen_route_cartesian_closed_form(P, ctx):
    """Fully sampled Cartesian: every eigenvalue of E^H E is N; R = E^H/(N + lam)."""
    n, lam = 12, 2.5
    enc = synth.Encoding(n, n, synth.cartesian_full(n, n))
    N = n * n
    info, spec, R, d, x = run(P, ctx, enc, P.FP64, lam, P.LAMBDA_ABS, P.TRUNC_KAPPA, 1.5)
    assert info["rank"] == N
    assert np.max(np.abs(spec - N)) <= 1e-12 * N
    Eh = oracle.encoding_matrix(enc).conj().T
    assert np.max(np.abs(R - Eh / (N + lam))) <= 1e-12 / (N + lam)


def test_eigen_route_refusals(P, ctx):
    enc = encoding("odd_c2")
    plan = P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED,
                        route=P.ROUTE_EIGEN)
    try:
        P.pinv_plan_wait(plan)
        d = torch.zeros((2, enc.M), dtype=torch.complex64, device="cuda")
        x = torch.zeros((2, enc.N), dtype=torch.complex64, device="cuda")
        with pytest.raises(P.PinvError) as ei:
            P.pinv_apply(ctx, plan, d, x, refine_steps=1)
        assert ei.value.status == P.ERR_INVALID
    finally:
        P.pinv_plan_release(plan)
    chol = P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    try:
        P.pinv_plan_wait(chol)
        out = torch.zeros((enc.N,), dtype=torch.float64, device="cuda")
        with pytest.raises(P.PinvError) as ei:
            P.pinv_spectrum(ctx, chol, out)
        assert ei.value.status == P.ERR_INVALID
    finally:
        P.pinv_plan_release(chol)
