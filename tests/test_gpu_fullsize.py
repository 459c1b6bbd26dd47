"""Parity at the workloads' full sizes, in the launch configuration the bench
times (FP32 plans, 1000/200 frames in one apply call, one refinement step).

* 32x32 single-coil radial (N=1024, M=2048), FP64: every stage against the full
  oracle (G within 1e-12 of max|G|, L^-1, R, the image, the SRF matrix and the
  white-noise matrix within 1e-9).
* 64x64, 8 coils (FP32 plan, as the bench times the metrics): the SRF map lies
  in (0, 1] up to the FP32 plan's error, the noise map is positive, and it
  equals the diagonal of the noise matrix within M * u32 (FP32 summation of
  M positive terms on the matrix side).
* 64x64, 8 coils, M=32768, 1000 frames and the 5-species + B0 workload
  (N=5120, M=49152, 200 frames): sampled Gram entries against the oracle's
  explicit E columns, within M * 2^-53 of max diag (the worst-case rounding of
  the oracle's own FP64 sum over M rows), and for sampled frames the
  normal-equation residual E^H(d - E x) - lam x formed by the oracle in FP64,
  for the FP32 plan, the FP32 factor-only plan (no R) and the FP64 plan.
  Its normwise backward error eta = ||r|| / ((max diag + lam) ||x||) is a
  necessary check only: it bounds the relative forward error from above
  only through kappa(G_l) (forward error <= kappa * eta), and max diag + lam
  underestimates ||G + lam I||, so a small eta alone does not prove a small
  forward error.  It must still be <= 1e-5 for refined FP32 and 1e-10 for
  FP64.  The forward error itself is checked against the FP64 GPU path, which
  the oracle validates element by element at the smaller shapes.  Frame data
  are seeded complex Gaussian draws (the residual identity holds for any data).
* 96x96, 16 coils, M=131072 (the precision-study workload), 500 frames: the
  same sampled Gram entries and oracle-formed residuals.  The oracle's
  forward and adjoint run coil by coil in threads (E^H r = sum_c E_c^H r_c,
  Eq. 11), since forming all 1.2e9 entries of E in one thread takes minutes.
"""
from concurrent.futures import ThreadPoolExecutor

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
    c = P.pinv_context_create(0)
    yield c
    P.pinv_context_destroy(c)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_radial32_every_stage(P, ctx):
    w = synth.radial_32x32_c1()
    enc = w.enc
    N, M = enc.N, enc.M
    ob = oracle.Build(enc, rel=w.rel_lambda)
    d0 = oracle.forward(enc, w.images)
    d = d0 + np.sqrt(np.mean(np.abs(d0) ** 2)) * 10 ** (-w.snr_db / 20) * w.noise
    x_ref = ob.reconstruct(d)
    R_ref = ob.recon_matrix()
    Li_ref = oracle.forward_substitution(ob.L, np.eye(N))
    plan = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP64, P.FLAG_UNCACHED)
    P.pinv_plan_wait(plan)
    G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    Li = torch.empty_like(G)
    R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
    P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li)
    P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
    dd = torch.from_numpy(d).cuda()
    x = torch.empty((1, N), dtype=torch.complex128, device="cuda")
    P.pinv_apply(ctx, plan, dd, x)
    torch.cuda.synchronize()
    assert np.max(np.abs(G.cpu().numpy() - ob.G)) <= 1e-12 * np.max(np.abs(ob.G))
    assert rel(np.tril(Li.cpu().numpy()), Li_ref) < 1e-9
    assert rel(R.cpu().numpy(), R_ref) < 1e-9
    assert rel(x.cpu().numpy(), x_ref) < 1e-9
    # image metrics (Eq. 9, Eq. 10) of the FP64 plan against the oracle's R
    E = oracle.encoding_matrix(enc)
    srf = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    X = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_srf(ctx, plan, srf, P.METRIC_FULL)
    P.pinv_noise(ctx, plan, X, mode=P.METRIC_FULL)
    torch.cuda.synchronize()
    assert rel(srf.cpu().numpy(), oracle.srf_matrix(R_ref, E)) < 1e-9
    assert rel(X.cpu().numpy(), oracle.noise_matrix(R_ref, np.eye(M))) < 1e-9
    P.pinv_plan_release(plan)
    # the FP32 path with one refinement step on the same input
    p32 = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    x32 = torch.empty((1, N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p32, dd.to(torch.complex64), x32, refine_steps=1)
    torch.cuda.synchronize()
    assert rel(x32.cpu().numpy().astype(np.complex128), x_ref) < 1e-5
    P.pinv_plan_release(p32)


def _coil_encoding(enc, c):
    return synth.Encoding(enc.nx, enc.ny, enc.k, t=enc.t,
                          coil=None if enc.coil is None else enc.coil[c:c + 1],
                          b0_hz=enc.b0_hz, species_hz=enc.species_hz,
                          voxels=getattr(enc, "voxels", None))


def oracle_residual(enc, d, xs, lam):
    """E^H (d - E x) - lam x for frames d [F, M] and images xs [F, N], formed by
    the oracle coil by coil (E_c = rows c*K .. c*K + K - 1; Eq. 11) in threads."""
    K, C = enc.K, enc.C

    def one(c):
        ec = _coil_encoding(enc, c)
        rc = d[:, c * K:(c + 1) * K] - oracle.forward(ec, xs)
        return oracle.adjoint(ec, rc)

    with ThreadPoolExecutor(max_workers=min(C, 16)) as ex:
        parts = list(ex.map(one, range(C)))
    return sum(parts) - lam * xs


def _sampled_checks(P, ctx, enc, rel_lam, F, frames, seed):
    N, M = enc.N, enc.M
    rng = np.random.default_rng(seed)
    d = synth.random_frames((F, M), rng)
    p32 = P.pinv_build(ctx, enc, rel_lam, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    p64 = P.pinv_build(ctx, enc, rel_lam, P.LAMBDA_REL_MEAN_DIAG, P.FP64, P.FLAG_UNCACHED)
    pfo = P.pinv_build(ctx, enc, rel_lam, P.LAMBDA_REL_MEAN_DIAG, P.FP32,
                       P.FLAG_UNCACHED | P.FLAG_NO_R)
    P.pinv_plan_wait(p32)
    P.pinv_plan_wait(p64)
    P.pinv_plan_wait(pfo)
    lam = P.pinv_plan_info_get(p32)["lambda_abs"]
    G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(p32, P.BUF_GRAM, G)
    d32 = torch.from_numpy(d.astype(np.complex64)).cuda()
    x32 = torch.empty((F, N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p32, d32, x32, refine_steps=1)
    xfo = torch.empty((F, N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, pfo, d32, xfo, refine_steps=1)
    d64 = torch.from_numpy(d).cuda()
    x64 = torch.empty((F, N), dtype=torch.complex128, device="cuda")
    P.pinv_apply(ctx, p64, d64, x64)
    torch.cuda.synchronize()
    # sampled Gram entries: diagonal, near-diagonal and random pairs
    a = np.concatenate([rng.integers(0, N, 96), np.arange(0, N, max(1, N // 32))])
    b = np.concatenate([rng.integers(0, N, 96), np.minimum(np.arange(0, N, max(1, N // 32)) + 1, N - 1)])
    a = np.concatenate([a, a[:32]])
    b = np.concatenate([b, a[:32]])
    g_ref = oracle.gram_entries(enc, a, b)
    g = G.cpu().numpy()[a, b]
    dmax = float(np.max(oracle.gram_entries(enc, a[-32:], a[-32:]).real))
    assert np.max(np.abs(g - g_ref)) <= M * 2.0 ** -53 * dmax
    # residual of the normal equations for sampled frames
    xs32 = x32[frames].cpu().numpy().astype(np.complex128)
    xs64 = x64[frames].cpu().numpy()
    xsfo = xfo[frames].cpu().numpy().astype(np.complex128)
    ds = d[frames]
    scale = dmax + lam
    nf = len(frames)
    stacked = np.concatenate([xs32, xs64, xsfo])
    r_all = oracle_residual(enc, np.concatenate([ds, ds, ds]), stacked, lam)
    for j, (xs, tol) in enumerate(((xs32, 1e-5), (xs64, 1e-10), (xsfo, 1e-5))):
        r = r_all[j * nf:(j + 1) * nf]
        eta = np.linalg.norm(r, axis=1) / (scale * np.linalg.norm(xs, axis=1))
        assert eta.max() <= tol, eta
    # and the device paths (R, factor-only, FP64) agree on every frame
    for x in (x32, xfo):
        e = (torch.linalg.vector_norm(x.to(torch.complex128) - x64, dim=1)
             / torch.linalg.vector_norm(x64, dim=1)).max().item()
        assert e < 1e-5, e
    P.pinv_plan_release(p32)
    P.pinv_plan_release(p64)
    P.pinv_plan_release(pfo)


def test_spiral64_c8_full_size_sampled(P, ctx):
    w = synth.spiral_64x64_c8(F=1)
    _sampled_checks(P, ctx, w.enc, w.rel_lambda, 1000, [0, 499, 999], seed=2024)


def test_spiral96_c16_full_size_sampled(P, ctx):
    """The precision-study workload at its full shape (N=9216, M=131072)."""
    w = synth.spiral_96x96_c16(F=1)
    _sampled_checks(P, ctx, w.enc, w.rel_lambda, 500, [0, 499], seed=3072)


def test_species5_full_size_sampled(P, ctx):
    w = synth.species5_32x32_c8(F=1)
    _sampled_checks(P, ctx, w.enc, w.rel_lambda, 200, [0, 199], seed=4048)


def test_spiral64_c8_metric_properties(P, ctx):
    w = synth.spiral_64x64_c8(F=1)
    enc = w.enc
    N = enc.N
    p = P.pinv_build(ctx, enc, w.rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    P.pinv_plan_wait(p)
    try:
        srf = torch.empty((N,), dtype=torch.complex64, device="cuda")
        nd = torch.empty((N,), dtype=torch.float32, device="cuda")
        X = torch.empty((N, N), dtype=torch.complex64, device="cuda")
        P.pinv_srf(ctx, p, srf, P.METRIC_DIAG)
        P.pinv_noise(ctx, p, nd, mode=P.METRIC_DIAG)
        P.pinv_noise(ctx, p, X, mode=P.METRIC_FULL)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(p)
    s = srf.cpu().numpy()
    assert np.all(s.real > 0) and np.all(s.real <= 1 + 1e-2)
    assert np.max(np.abs(s.imag)) < 1e-2
    n = nd.cpu().numpy().astype(np.float64)
    Xd = np.diagonal(X.cpu().numpy()).real.astype(np.float64)
    assert np.all(n > 0)
    # the map sums |R[n][m]|^2 in FP64; the matrix diagonal is an FP32 MFMA sum
    # of the same M positive terms, within the recursive-summation bound M * u32
    tol = enc.M * 2.0 ** -24
    assert abs(n.sum() - Xd.sum()) <= tol * n.sum()
    assert np.max(np.abs(n - Xd) / n) <= tol
