"""Fewer samples than unknowns (Sec. 2.2): the build takes the right
pseudoinverse R = E^H (E E^H + lam I)^-1 through the M x M samples' Gram,
checked against the FP64 oracle's RightBuild (its own pins tie it to the left
route with a shift and to the SVD pseudoinverse at zero shift).

Tolerances: FP64 plans 1e-9 relative with a shift (kappa(E E^H + lam I) <= 1e5
here) and kappa * 1e-14 at zero shift; FP32 plans kappa * 1e-6, as for the
N x N route, and 1e-6 after two refinement steps (made on the sample side,
with y held in FP64, so the limit is the FP32 rounding of the image, ~6e-8).  Shapes are ragged against the 64-wide FP64 and 128 x 64 FP32
tiles, with the generated loaders' aligned (nx, K multiples of 8) and general
paths, and with species and off-resonance factors.
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


CASES = {
    "aligned_c2": dict(seed=131, nx=16, ny=12, C=2, K=40, F=3),                       # M 80 < N 192
    "general_c3": dict(seed=132, nx=13, ny=11, C=3, K=29, F=2),                       # M 87 < N 143
    "species_b0": dict(seed=133, nx=12, ny=8, C=2, K=48, F=2, species=[0.0, 150.0], b0=True),
    # several 64-wide factor blocks (the look-ahead's second part runs) and
    # several tiles in every grid of the right-pseudoinverse products
    "multiblock_c3": dict(seed=134, nx=40, ny=36, C=3, K=200, F=2),                   # M 600 < N 1440
    "multiblock_c2": dict(seed=135, nx=30, ny=26, C=2, K=171, F=2),                   # M 342 < N 780
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def build(P, ctx, enc, prec, lam, mode):
    p = P.pinv_build(ctx, enc, lam, mode, prec, P.FLAG_UNCACHED)
    P.pinv_plan_wait(p)
    return p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_right_pinv_matches_oracle(P, ctx, name, prec):
    w = synth.small_case(**CASES[name])
    enc, N, M = w.enc, w.enc.N, w.enc.M
    assert M < N
    ob = oracle.RightBuild(enc, rel=1e-3)
    ev = np.linalg.eigvalsh(ob.Gr + ob.lam * np.eye(M))
    kappa = ev[-1] / ev[0]
    pr, cdt = (P.FP64, np.complex128) if prec == "fp64" else (P.FP32, np.complex64)
    p = build(P, ctx, enc, pr, 1e-3, P.LAMBDA_REL_MEAN_DIAG)
    try:
        info = P.pinv_plan_info_get(p)
        assert info["gram_order"] == M and info["has_r"]
        assert abs(info["lambda_abs"] - ob.lam) <= 1e-12 * ob.lam
        R = torch.empty((N, M), dtype=torch.complex128 if prec == "fp64" else torch.complex64,
                        device="cuda")
        P.pinv_plan_copy_buffer(p, P.BUF_R, R)
        G = torch.empty((M, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(p, P.BUF_GRAM, G)
        rng = np.random.default_rng(CASES[name]["seed"])
        d = rng.standard_normal((5, M)) + 1j * rng.standard_normal((5, M))
        dd = torch.from_numpy(d.astype(cdt)).cuda()
        x = torch.full((5, N), float("nan"), dtype=dd.dtype, device="cuda")
        torch.cuda.synchronize()
        P.pinv_apply(ctx, p, dd, x)
        # refinement on the sample side: y = G'^-1 d refined against the FP64 G', x = E^H y
        x2 = torch.full((5, N), float("nan"), dtype=dd.dtype, device="cuda")
        P.pinv_apply(ctx, p, dd, x2, refine_steps=2)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(p)
    e_x2 = rel(x2.cpu().numpy().astype(np.complex128), ob.reconstruct(d))
    print(f"{name} {prec}: refined (2 steps) x {e_x2:.2e}")
    assert e_x2 < (1e-9 if prec == "fp64" else 1e-6)
    tol = 1e-9 if prec == "fp64" else kappa * 1e-6
    g = G.cpu().numpy()
    assert np.max(np.abs(np.tril(g) - np.tril(ob.Gr))) <= 1e-12 * np.max(np.abs(ob.Gr))
    R_ref = ob.recon_matrix()
    e_r = rel(R.cpu().numpy().astype(np.complex128), R_ref)
    if prec == "fp64":   # element by element as well
        e_entry = np.max(np.abs(R.cpu().numpy() - R_ref)) / np.max(np.abs(R_ref))
        assert e_entry < 1e-9, e_entry
    e_x = rel(x.cpu().numpy().astype(np.complex128), ob.reconstruct(d))
    print(f"{name} {prec}: kappa={kappa:.3g} R {e_r:.2e} x {e_x:.2e}")
    assert e_r < tol and e_x < tol


def test_right_pinv_minimum_norm_at_zero_shift(P, ctx):
    """lambda = 0: the minimum-norm solution; R E R = R and E R = I to FP64
    accuracy scaled by the condition number of E E^H."""
    w = synth.small_case(**CASES["aligned_c2"])
    enc, N, M = w.enc, w.enc.N, w.enc.M
    ob = oracle.RightBuild(enc, lam=0.0)
    ev = np.linalg.eigvalsh(ob.Gr)
    kappa = ev[-1] / ev[0]
    p = build(P, ctx, enc, P.FP64, 0.0, P.LAMBDA_ABS)
    try:
        R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(p, P.BUF_R, R)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(p)
    R = R.cpu().numpy()
    E = oracle.encoding_matrix(enc)
    print(f"kappa(E E^H) = {kappa:.3g}")
    assert rel(R, ob.recon_matrix()) < max(1e-9, kappa * 1e-14)
    assert np.linalg.norm(E @ R - np.eye(M)) < max(1e-9, kappa * 1e-14) * np.sqrt(M)


def test_overdiscretised_grid(P, ctx):
    """Overdiscretisation: a 24 x 20 grid (N = 480) over the k-space extent of a
    12 x 10 one, 2 coils x 100 samples (M = 200 < N), takes the right
    pseudoinverse; FP64 image and R against the oracle's RightBuild."""
    rng = np.random.default_rng(141)
    k = synth.vd_spiral(12, 100)
    enc = synth.Encoding(24, 20, k, coil=synth.coil_maps(24, 20, 2, rng))
    N, M = enc.N, enc.M
    ob = oracle.RightBuild(enc, rel=1e-3)
    p = build(P, ctx, enc, P.FP64, 1e-3, P.LAMBDA_REL_MEAN_DIAG)
    d = rng.standard_normal((4, M)) + 1j * rng.standard_normal((4, M))
    try:
        assert P.pinv_plan_info_get(p)["gram_order"] == M
        R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(p, P.BUF_R, R)
        dd = torch.from_numpy(d).cuda()
        x = torch.empty((4, N), dtype=torch.complex128, device="cuda")
        P.pinv_apply(ctx, p, dd, x)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(p)
    assert rel(R.cpu().numpy(), ob.recon_matrix()) < 1e-9
    assert rel(x.cpu().numpy(), ob.reconstruct(d)) < 1e-9


def test_right_pinv_refused_options(P, ctx):
    enc = synth.small_case(**CASES["aligned_c2"]).enc
    for prec, flags, want in ((P.BF16X3, P.FLAG_UNCACHED, P.ERR_UNSUPPORTED),
                              (P.FP32, P.FLAG_UNCACHED | P.FLAG_NO_R, P.ERR_INVALID)):
        with pytest.raises(P.PinvError) as ei:
            P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, prec, flags)
        assert ei.value.status == want
