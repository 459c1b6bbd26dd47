"""Voxel masks (Sec. 3.1 and Sec. 4.4: unknowns restricted to a circular field
of view or to voxels above a signal threshold) on the HIP path, against the
FP64 oracle restricted to the same voxels.

The masked encodings are ragged against every tile (N = S * nvox is no multiple
of 64) and their voxel lists break the image-row alignment the row-generated
loaders otherwise use (the wide case at 64 x 48, 2395 unknowns, spans many
tiles).  Bars as for the unmasked parity tests: FP64 plans 1e-9
relative (R and L^-1 element by element, the Gram within 1e-12 of max|G|),
FP32 plans 1e-5 after two refinement steps.
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


def masked(w, vox):
    e = w.enc
    return synth.Encoding(e.nx, e.ny, e.k, t=e.t, coil=e.coil, b0_hz=e.b0_hz,
                          species_hz=e.species_hz, voxels=vox)


def frame_rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def max_rel_entry(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def case(name):
    if name == "circle_c3":       # circular field of view, 3 coils (PSF Gram)
        w = synth.small_case(seed=201, nx=26, ny=22, C=3, K=900, F=4)
        return w, masked(w, synth.circular_mask(26, 22))
    if name == "threshold_c2":    # voxels above 30% of the phantom's peak (PSF Gram)
        w = synth.small_case(seed=202, nx=24, ny=24, C=2, K=1100, F=3)
        return w, masked(w, synth.threshold_mask(w.images[0], 0.3))
    if name == "wide_disc_c2":    # rows up to 64 voxels wide, wider than a 32-column
        # chunk: several tiles in each dimension and chunks within and across rows
        w = synth.small_case(seed=204, nx=64, ny=48, C=2, K=2600, F=3)
        return w, masked(w, synth.circular_mask(64, 48))
    if name == "circle_species_b0":   # two species and off-resonance (MFMA Gram)
        w = synth.small_case(seed=203, nx=16, ny=16, C=2, K=700, F=3, species=[0.0, 150.0], b0=True)
        return w, masked(w, synth.circular_mask(16, 16, 0.9))
    raise KeyError(name)


_cache = {}


def oracle_case(name):
    if name not in _cache:
        w, enc = case(name)
        rng = np.random.default_rng(7)
        d = synth.random_frames((3, enc.M), rng)
        b = oracle.Build(enc, rel=1e-3)
        _cache[name] = dict(enc=enc, d=d, b=b, x=b.reconstruct(d), R=b.recon_matrix(),
                            Linv=oracle.forward_substitution(b.L, np.eye(enc.N)))
    return _cache[name]


NAMES = ["circle_c3", "threshold_c2", "wide_disc_c2", "circle_species_b0"]


@pytest.mark.parametrize("name", NAMES)
def test_masked_fp64_plan_matches_oracle(P, ctx, name):
    o = oracle_case(name)
    enc, N, M = o["enc"], o["enc"].N, o["enc"].M
    assert N % 64 != 0
    plan = P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP64, P.FLAG_UNCACHED)
    try:
        P.pinv_plan_wait(plan)
        info = P.pinv_plan_info_get(plan)
        assert info["N"] == N and abs(info["lambda_abs"] - o["b"].lam) <= 1e-12 * o["b"].lam
        G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
        Li = torch.empty_like(G)
        R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
        P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li)
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        d = torch.from_numpy(o["d"]).cuda()
        x = torch.empty((3, N), dtype=torch.complex128, device="cuda")
        P.pinv_apply(ctx, plan, d, x)
        # forward model of the masked encoding (Eq. 1)
        dd = torch.empty((3, M), dtype=torch.complex128, device="cuda")
        P.pinv_forward(ctx, plan, torch.from_numpy(o["x"]).cuda(), dd)
        srf = torch.empty((N,), dtype=torch.complex128, device="cuda")
        P.pinv_srf(ctx, plan, srf, P.METRIC_DIAG)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    assert np.max(np.abs(G.cpu().numpy() - o["b"].G)) <= 1e-12 * np.max(np.abs(o["b"].G))
    assert max_rel_entry(np.tril(Li.cpu().numpy()), o["Linv"]) < 1e-9
    assert max_rel_entry(R.cpu().numpy(), o["R"]) < 1e-9
    assert frame_rel(x.cpu().numpy(), o["x"]).max() < 1e-9
    assert frame_rel(dd.cpu().numpy(), oracle.forward(enc, o["x"])).max() < 1e-12
    srf_ref = np.diagonal(oracle.srf_matrix(o["R"], oracle.encoding_matrix(enc)))
    assert max_rel_entry(srf.cpu().numpy(), srf_ref) < 1e-9


@pytest.mark.parametrize("name", NAMES)
def test_masked_fp32_plan_refined(P, ctx, name):
    """FP32 plans with a mask: the row-generated loaders take the masked
    (unaligned) path in W; images within 1e-5 after two refinement steps, also
    for the factor-only plan."""
    o = oracle_case(name)
    enc, N = o["enc"], o["enc"].N
    d = torch.from_numpy(o["d"].astype(np.complex64)).cuda()
    for flags in (P.FLAG_UNCACHED, P.FLAG_UNCACHED | P.FLAG_NO_R):
        plan = P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP32, flags)
        try:
            P.pinv_plan_wait(plan)
            x = torch.empty((3, N), dtype=torch.complex64, device="cuda")
            P.pinv_apply(ctx, plan, d, x, refine_steps=2)
            torch.cuda.synchronize()
        finally:
            P.pinv_plan_release(plan)
        e = frame_rel(x.cpu().numpy().astype(np.complex128), o["x"]).max()
        print(f"{name} flags {flags}: refined err {e:.2e}")
        assert e < 1e-5


def test_masked_gram_forms_agree(P, ctx):
    """The PSF Gram and the MFMA Gram of a masked encoding, both against the
    oracle's masked Gram."""
    o = oracle_case("circle_c3")
    enc, N = o["enc"], o["enc"].N
    for g in (P.GRAM_PSF, P.GRAM_SHARED):
        plan = P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP64, P.FLAG_UNCACHED,
                            gram=g)
        try:
            P.pinv_plan_wait(plan)
            G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
            P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
            torch.cuda.synchronize()
        finally:
            P.pinv_plan_release(plan)
        assert np.max(np.abs(G.cpu().numpy() - o["b"].G)) <= 1e-12 * np.max(np.abs(o["b"].G))
