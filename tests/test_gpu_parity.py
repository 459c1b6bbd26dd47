"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Shapes span several 64/128 tiles with ragged tails (N = 480, 288, 640, 256;
M = 2100, 1000, 1408, 1024), include the species and off-resonance factors, and
cover both the general and the aligned chunk paths of the generated loaders.  Tolerances:

* FP64 plans: every stage within 1e-9 relative (Frobenius) of the oracle; the
  FP64 forward error of the Cholesky route is ~kappa(G_l) * 1e-16 with
  kappa <= 1e4 here.
* Default Gram (FP64 F^H F times the coil cross-products, exact because every
  coil shares the trajectory): within 1e-12 of max|G| for every plan.
* Full-M Gram in FP32 (PINV_FLAG_GRAM_FULL): within 2048 * u32 = 1.2e-4 of
  max|G|: each entry is a sum of FP32 products accumulated in FP32 over
  segments of 2048 rows (then carried in FP64), and a sum of L terms bounded
  by max|G| carries at most about L*u32*max|G| of rounding.
* FP32 plans: images after two refinement steps within 1e-5 (the target for
  the FP32 path); before refinement within kappa(G_l) * 1e-6.
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def frame_rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def max_rel_entry(a, b):
    """Largest entrywise difference relative to the largest reference entry."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


CASES = {
    "ragged_c3": dict(seed=101, nx=24, ny=20, C=3, K=700, F=5),
    "species_b0": dict(seed=102, nx=12, ny=12, C=2, K=500, F=4, species=[0.0, 150.0], b0=True),
    # nx and K multiples of 32: the generated loaders' aligned chunk paths (FP32,
    # FP64 and BF16-split tiles), still ragged against the 64/128 tiles (N = 640)
    "aligned_c2": dict(seed=103, nx=32, ny=20, C=2, K=704, F=3),
    "aligned_species_b0": dict(seed=104, nx=16, ny=8, C=2, K=512, F=3, species=[0.0, 150.0],
                               b0=True),
}

# cases used by single tests only (not every CASES-parametrised test)
EXTRA_CASES = {
    # M = 10400 >= 8192: the row apply's contraction is sliced over the XCDs
    "long_c4": dict(seed=105, nx=24, ny=20, C=4, K=2600, F=2),
    # M = 9003, odd: the streamed apply's 8-byte loads, a partial last chunk
    "long_odd": dict(seed=106, nx=22, ny=19, C=3, K=3001, F=2),
}

_oracle_cache = {}


def oracle_case(name):
    if name not in _oracle_cache:
        kw = dict(CASES[name] if name in CASES else EXTRA_CASES[name])
        w = synth.small_case(**kw)
        b = oracle.Build(w.enc, rel=1e-3)
        d0 = oracle.forward(w.enc, w.images)
        sig = np.sqrt(np.mean(np.abs(d0) ** 2))
        d = d0 + sig * 10 ** (-30 / 20) * w.noise
        x = b.reconstruct(d)
        Lo_inv = oracle.forward_substitution(b.L, np.eye(b.L.shape[0]))
        R = b.recon_matrix()
        ev = np.linalg.eigvalsh(b.G + b.lam * np.eye(b.G.shape[0]))
        _oracle_cache[name] = dict(w=w, b=b, d=d, x=x, Linv=Lo_inv, R=R, kappa=ev[-1] / ev[0])
    return _oracle_cache[name]


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


def build(P, ctx, enc, prec, flags=0, lam=1e-3, mode=None, **kw):
    mode = P.LAMBDA_REL_MEAN_DIAG if mode is None else mode
    plan = P.pinv_build(ctx, enc, lam, mode, prec, flags, **kw)
    P.pinv_plan_wait(plan)
    return plan


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_stages_match_oracle(P, ctx, name):
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    plan = build(P, ctx, enc, P.FP64, flags=P.FLAG_KEEP_GRAM)
    info = P.pinv_plan_info_get(plan)
    assert info["N"] == N and info["M"] == M
    assert abs(info["lambda_abs"] - o["b"].lam) <= 1e-12 * o["b"].lam
    G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
    Li = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li)
    R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
    torch.cuda.synchronize()
    G = np.tril(G.cpu().numpy())
    Go = np.tril(o["b"].G)
    assert np.max(np.abs(G - Go)) <= 1e-12 * np.max(np.abs(Go))
    assert rel(np.tril(Li.cpu().numpy()), o["Linv"]) < 1e-9
    assert rel(R.cpu().numpy(), o["R"]) < 1e-9
    # element by element, so a mis-indexed ragged tail tile of small entries fails too
    assert max_rel_entry(np.tril(Li.cpu().numpy()), o["Linv"]) < 1e-9
    assert max_rel_entry(R.cpu().numpy(), o["R"]) < 1e-9
    d = to_dev(o["d"], np.complex128)
    x = torch.empty((d.shape[0], N), dtype=torch.complex128, device="cuda")
    P.pinv_apply(ctx, plan, d, x)
    torch.cuda.synchronize()
    err = frame_rel(x.cpu().numpy(), o["x"])
    assert err.max() < 1e-9, err
    P.pinv_plan_release(plan)


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_path_matches_oracle(P, ctx, name):
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    plan = build(P, ctx, enc, P.FP32, flags=P.FLAG_KEEP_GRAM)
    G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
    torch.cuda.synchronize()
    G = np.tril(G.cpu().numpy())
    Go = np.tril(o["b"].G)
    gerr = np.max(np.abs(G - Go)) / np.max(np.abs(Go))
    assert gerr < 1e-12, gerr
    d = to_dev(o["d"], np.complex64)
    x0 = torch.empty((d.shape[0], N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, plan, d, x0, refine_steps=0)
    x2 = torch.empty_like(x0)
    P.pinv_apply(ctx, plan, d, x2, refine_steps=2)
    torch.cuda.synchronize()
    e0 = frame_rel(x0.cpu().numpy().astype(np.complex128), o["x"])
    e2 = frame_rel(x2.cpu().numpy().astype(np.complex128), o["x"])
    print(f"{name}: kappa={o['kappa']:.3g} gram_err={gerr:.2e} err0={e0.max():.2e} err2={e2.max():.2e}")
    assert e0.max() < o["kappa"] * 1e-6
    assert e2.max() < 1e-5
    P.pinv_plan_release(plan)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_full_gram_matches_oracle(P, ctx, name, prec):
    """The Gram over all M rows in the plan's precision (no shared-trajectory shortcut)."""
    o = oracle_case(name)
    enc, N = o["w"].enc, o["w"].enc.N
    p = P.FP64 if prec == "fp64" else P.FP32
    plan = build(P, ctx, enc, p, flags=P.FLAG_KEEP_GRAM | P.FLAG_GRAM_FULL)
    G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
    d = to_dev(o["d"], np.complex128 if prec == "fp64" else np.complex64)
    x = torch.empty((d.shape[0], N), dtype=d.dtype, device="cuda")
    P.pinv_apply(ctx, plan, d, x, refine_steps=0 if prec == "fp64" else 2)
    torch.cuda.synchronize()
    G = np.tril(G.cpu().numpy())
    Go = np.tril(o["b"].G)
    gerr = np.max(np.abs(G - Go)) / np.max(np.abs(Go))
    assert gerr < (1e-12 if prec == "fp64" else 2048 * 2.0 ** -24), gerr
    err = frame_rel(x.cpu().numpy().astype(np.complex128), o["x"]).max()
    assert err < (1e-9 if prec == "fp64" else 1e-5), err
    P.pinv_plan_release(plan)


@pytest.mark.parametrize("name", list(CASES))
def test_bf16x3_path_matches_oracle(P, ctx, name):
    """BF16-split products (hi*hi + hi*lo + lo*hi, ~2^-16 per product) for W, R and the
    apply; FP64 factor; refinement with FP64 residuals and the FP32 factor.  Targets:
    before refinement within kappa * 1e-4, after two steps within 3e-3 (the BF16-split
    target) -- in practice FP32-level since the correction uses the FP32 factor."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    plan = build(P, ctx, enc, P.BF16X3)
    d = to_dev(o["d"], np.complex64)
    x0 = torch.empty((d.shape[0], N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, plan, d, x0, refine_steps=0)
    x2 = torch.empty_like(x0)
    P.pinv_apply(ctx, plan, d, x2, refine_steps=2)
    R = torch.full((N, M), float("nan"), dtype=torch.complex64, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_R, R)    # unpacked from the split-packed R
    torch.cuda.synchronize()
    e0 = frame_rel(x0.cpu().numpy().astype(np.complex128), o["x"])
    e2 = frame_rel(x2.cpu().numpy().astype(np.complex128), o["x"])
    eR = max_rel_entry(R.cpu().numpy().astype(np.complex128), o["R"])
    print(f"{name}: bf16x3 err0={e0.max():.2e} err2={e2.max():.2e} R {eR:.2e}")
    assert eR < o["kappa"] * 1e-4
    assert e0.max() < o["kappa"] * 1e-4
    assert e2.max() < 3e-3
    P.pinv_plan_release(plan)


@pytest.mark.parametrize("name", ["ragged_c3", "aligned_c2"])
def test_bf16x3_apply_paths(P, ctx, name):
    """A BF16X3 plan keeps R split into bf16 hi/lo planes (rows padded to a
    multiple of 32 columns: M = 2100 leaves a ragged 8-group and padding).
    Its applies of at most 8 frames stream those rows and multiply by hi + lo
    in FP32; more frames split the data too and run BF16x3 tiles.  Both
    against the plan's own R (copied out as complex64, so exact) applied in
    FP64: rows within 1e-5 (FP32 sums), tiles within 2e-4 (the data's split
    adds ~2^-16 per product); and against the oracle's R at kappa * 1e-4."""
    o = oracle_case(name)
    w, N, M = o["w"], o["w"].enc.N, o["w"].enc.M
    rng = np.random.default_rng(37)
    Fmax = 150
    d = rng.standard_normal((Fmax, M)) + 1j * rng.standard_normal((Fmax, M))
    d = d.astype(np.complex64).astype(np.complex128)
    plan = build(P, ctx, w.enc, P.BF16X3, flags=P.FLAG_UNCACHED)
    try:
        R = torch.full((N, M), float("nan"), dtype=torch.complex64, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        torch.cuda.synchronize()
        Rp = R.cpu().numpy().astype(np.complex128)
        assert np.all(np.isfinite(Rp))
        x_own, x_or = d @ Rp.T, d @ o["R"].T
        for F in (1, 3, 8, 9, 40, Fmax):
            dd = to_dev(d[:F], np.complex64)
            x = torch.full((F, N), float("nan"), dtype=torch.complex64, device="cuda")
            torch.cuda.synchronize()
            P.pinv_apply(ctx, plan, dd, x)
            torch.cuda.synchronize()
            xg = x.cpu().numpy().astype(np.complex128)
            e_own, e_or = frame_rel(xg, x_own[:F]).max(), frame_rel(xg, x_or[:F]).max()
            print(f"{name} F={F}: vs own R {e_own:.2e}, vs oracle R {e_or:.2e}")
            assert e_own < (1e-5 if F <= 8 else 2e-4), (F, e_own)
            assert e_or < o["kappa"] * 1e-4, (F, e_or)
    finally:
        P.pinv_plan_release(plan)


@pytest.mark.parametrize("name", ["ragged_c3", "aligned_c2"])
def test_factor_on_a_side_stream(P, ctx, name):
    """A build issued on a non-default stream runs the factorisation's bulk
    trailing updates on the library's CU-restricted look-ahead stream (builds on
    the null stream use an unrestricted one); L^-1 and R must match the oracle
    either way."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = P.pinv_build(ctx, enc, o["w"].rel_lambda, P.LAMBDA_REL_MEAN_DIAG, P.FP64,
                            P.FLAG_UNCACHED, stream=side)
        P.pinv_plan_wait(plan)
        Li = torch.empty((N, N), dtype=torch.complex128, device="cuda")
        R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li, stream=side)
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R, stream=side)
        side.synchronize()
    P.pinv_plan_release(plan)
    assert rel(np.tril(Li.cpu().numpy()), o["Linv"]) < 1e-9
    assert rel(R.cpu().numpy(), o["R"]) < 1e-9


def test_single_coil_spiral_factor(P, ctx):
    """Single-coil spirals of the serving mix (K = 2N): the Gram is numerically
    rank deficient and its diagonal blocks are ill-conditioned (a regression case
    for the diagonal-block elimination).  32x32: L^-1 against the oracle; 64x64:
    the build succeeds and the FP64 images satisfy the normal equations
    (backward error <= 1e-10, residual formed by the oracle)."""
    enc = synth.serving_encoding(32, 1, 3)
    N = enc.N
    ob = oracle.Build(enc, rel=1e-3)
    Lo_inv = oracle.forward_substitution(ob.L, np.eye(N))
    plan = build(P, ctx, enc, P.FP64)
    Li = torch.empty((N, N), dtype=torch.complex128, device="cuda")
    P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li)
    torch.cuda.synchronize()
    assert rel(np.tril(Li.cpu().numpy()), Lo_inv) < 1e-9
    P.pinv_plan_release(plan)
    enc = synth.serving_encoding(64, 1, 9)
    plan = build(P, ctx, enc, P.FP64)
    lam = P.pinv_plan_info_get(plan)["lambda_abs"]
    d = synth.random_frames((2, enc.M), np.random.default_rng(9))
    x = torch.empty((2, enc.N), dtype=torch.complex128, device="cuda")
    P.pinv_apply(ctx, plan, to_dev(d, np.complex128), x)
    torch.cuda.synchronize()
    xs = x.cpu().numpy()
    r = oracle.adjoint(enc, d - oracle.forward(enc, xs)) - lam * xs
    eta = np.linalg.norm(r, axis=1) / ((enc.K + lam) * np.linalg.norm(xs, axis=1))
    assert eta.max() < 1e-10, eta
    P.pinv_plan_release(plan)


def test_cartesian_lambda0_inverse_dft(P, ctx):
    n = 16
    enc = synth.Encoding(n, n, synth.cartesian_full(n, n))
    plan = P.pinv_build(ctx, enc, 0.0, P.LAMBDA_ABS, P.FP64)
    P.pinv_plan_wait(plan)
    d = synth.unit_complex_noise((3, n * n), np.random.default_rng(9))
    dd = to_dev(d, np.complex128)
    x = torch.empty((3, n * n), dtype=torch.complex128, device="cuda")
    P.pinv_apply(ctx, plan, dd, x)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    for f in range(3):
        ref = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(d[f].reshape(n, n)))).ravel()
        assert rel(x[f], ref) < 1e-12
    P.pinv_plan_release(plan)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_matches_oracle(P, ctx, prec):
    o = oracle_case("species_b0")
    enc = o["w"].enc
    p = P.FP64 if prec == "fp64" else P.FP32
    dt = np.complex128 if prec == "fp64" else np.complex64
    plan = build(P, ctx, enc, p)
    x = to_dev(o["w"].images, dt)
    d = torch.empty((x.shape[0], enc.M), dtype=x.dtype, device="cuda")
    P.pinv_forward(ctx, plan, x, d)
    torch.cuda.synchronize()
    ref = oracle.forward(enc, o["w"].images)
    err = frame_rel(d.cpu().numpy().astype(np.complex128), ref).max()
    assert err < (1e-12 if prec == "fp64" else 2e-6), err
    P.pinv_plan_release(plan)


def test_not_positive_definite_is_reported(P, ctx):
    # four samples at k = 0 on a 2x2 grid: E is all ones, G = 4*ones, rank 1
    enc = synth.Encoding(2, 2, np.zeros((4, 2)))
    for prec in (P.FP64, P.FP32):
        plan = P.pinv_build(ctx, enc, 0.0, P.LAMBDA_ABS, prec)
        st = P.pinv_plan_wait_status(plan)
        assert st == P.ERR_NOT_PD
        assert "column 1" in P.pinv_last_error()
        P.pinv_plan_release(plan)


def test_invalid_arguments(P, ctx):
    # M < N with lambda = 0 takes the right pseudoinverse; ten identical samples
    # (k = 0) make E E^H rank one, which the factorisation reports
    enc = synth.Encoding(8, 8, np.zeros((10, 2)))
    p = P.pinv_build(ctx, enc, 0.0, P.LAMBDA_ABS, P.FP64, P.FLAG_UNCACHED)
    try:
        with pytest.raises(P.PinvError) as ei:
            P.pinv_plan_wait(p)
        assert ei.value.status == P.ERR_NOT_PD
    finally:
        P.pinv_plan_release(p)
    with pytest.raises(P.PinvError):
        P.pinv_build(ctx, enc, -1.0, P.LAMBDA_ABS, P.FP64)


def test_zero_frames_and_grouped_equals_single(P, ctx):
    o1, o2 = oracle_case("ragged_c3"), oracle_case("species_b0")
    p1 = build(P, ctx, o1["w"].enc, P.FP32)
    p2 = build(P, ctx, o2["w"].enc, P.FP32)
    d1, d2 = to_dev(o1["d"], np.complex64), to_dev(o2["d"], np.complex64)
    x1 = torch.zeros((d1.shape[0], o1["w"].enc.N), dtype=torch.complex64, device="cuda")
    x2 = torch.zeros((d2.shape[0], o2["w"].enc.N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p1, d1, x1)
    P.pinv_apply(ctx, p2, d2, x2)
    g1, g2 = torch.zeros_like(x1), torch.zeros_like(x2)
    P.pinv_apply_grouped(ctx, [(p1, d1, g1), (p2, d2, g2)])
    e = torch.empty((0, o1["w"].enc.M), dtype=torch.complex64, device="cuda")
    ex = torch.empty((0, o1["w"].enc.N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p1, e, ex)
    torch.cuda.synchronize()
    assert torch.equal(g1, x1) and torch.equal(g2, x2)
    # a frame's result does not depend on the values of the other frames (the
    # path follows from F, N and M, so the batch keeps its size; every path
    # is covered: rows at F = 1 and 2, streamed at 3 to 32, tiles at 40)
    gen = torch.Generator(device="cuda").manual_seed(7)
    for F in (1, 2, 3, 8, 32, 40):
        d = torch.randn((F, o1["w"].enc.M), dtype=torch.complex64, device="cuda", generator=gen)
        d_alt = torch.randn((F, o1["w"].enc.M), dtype=torch.complex64, device="cuda", generator=gen)
        f = F // 2
        d_alt[f] = d[f]
        x, x_alt = (torch.zeros((F, o1["w"].enc.N), dtype=torch.complex64, device="cuda")
                    for _ in range(2))
        P.pinv_apply(ctx, p1, d, x)
        P.pinv_apply(ctx, p1, d_alt, x_alt)
        torch.cuda.synchronize()
        assert torch.equal(x[f], x_alt[f]), F
    P.pinv_plan_release(p1)
    P.pinv_plan_release(p2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_factor_only_plan_matches_oracle(P, ctx, name, prec):
    """A plan built with FLAG_NO_R keeps L^-1 and the Gram but no R; its applies
    solve x = L^-H L^-1 (E^H d) with E regenerated per tile, which equals R d.
    Same bars as the R path: FP64 1e-9; FP32 kappa * 1e-6 unrefined and 1e-5
    after two refinement steps.  The metrics need R and are refused."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    pr = P.FP64 if prec == "fp64" else P.FP32
    cdt = np.complex128 if prec == "fp64" else np.complex64
    plan = build(P, ctx, enc, pr, flags=P.FLAG_NO_R | P.FLAG_UNCACHED)
    full = build(P, ctx, enc, pr, flags=P.FLAG_UNCACHED)
    try:
        info, finfo = P.pinv_plan_info_get(plan), P.pinv_plan_info_get(full)
        assert not info["has_r"] and finfo["has_r"]
        assert info["stage_ms"][2] == 0.0 and info["stage_ms"][3] == 0.0
        assert info["device_bytes"] < finfo["device_bytes"]
        assert info["key"] != finfo["key"]
        d = to_dev(o["d"], cdt)
        F = d.shape[0]
        x0 = torch.full((F, N), float("nan"), dtype=d.dtype, device="cuda")
        x2 = torch.full((F, N), float("nan"), dtype=d.dtype, device="cuda")
        torch.cuda.synchronize()
        P.pinv_apply(ctx, plan, d, x0, refine_steps=0)
        P.pinv_apply(ctx, plan, d, x2, refine_steps=2)
        # grouped with an R plan: each item as alone
        g0, g1 = torch.zeros_like(x0), torch.zeros_like(x0)
        r0 = torch.zeros_like(x0)
        P.pinv_apply(ctx, full, d, r0)
        P.pinv_apply_grouped(ctx, [(full, d, g0), (plan, d, g1)])
        torch.cuda.synchronize()
        assert torch.equal(g1, x0) and torch.equal(g0, r0)
        e0 = frame_rel(x0.cpu().numpy().astype(np.complex128), o["x"])
        e2 = frame_rel(x2.cpu().numpy().astype(np.complex128), o["x"])
        print(f"{name} {prec}: kappa={o['kappa']:.3g} err0={e0.max():.2e} err2={e2.max():.2e}")
        if prec == "fp64":
            assert e0.max() < 1e-9 and e2.max() < 1e-9
        else:
            assert e0.max() < o["kappa"] * 1e-6
            assert e2.max() < 1e-5
        out = torch.zeros((N,), dtype=d.dtype, device="cuda")
        with pytest.raises(P.PinvError) as ei:
            P.pinv_srf(ctx, plan, out, P.METRIC_DIAG)
        assert ei.value.status == P.ERR_UNSUPPORTED
        with pytest.raises(P.PinvError) as ei:
            P.pinv_noise(ctx, plan, out.real.contiguous(), mode=P.METRIC_DIAG)
        assert ei.value.status == P.ERR_UNSUPPORTED
        Rb = torch.zeros((N, M), dtype=d.dtype, device="cuda")
        with pytest.raises(P.PinvError) as ei:
            P.pinv_plan_copy_buffer(plan, P.BUF_R, Rb)
        assert ei.value.status == P.ERR_INVALID
    finally:
        P.pinv_plan_release(plan)
        P.pinv_plan_release(full)


def test_factor_only_rejects_bf16x3(P, ctx):
    enc = oracle_case("species_b0")["w"].enc
    with pytest.raises(P.PinvError) as ei:
        P.pinv_build(ctx, enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.BF16X3, P.FLAG_NO_R)
    assert ei.value.status == P.ERR_INVALID


def test_release_is_ordered_after_pending_applies(P, ctx):
    """Releasing a plan does not wait on the host; its buffers go back to the
    plan pool behind every apply enqueued on it.  An apply still queued on a
    side stream when the plan is released, with a new build of the same size
    issued right after, must give the same image bit for bit."""
    encs = [synth.serving_encoding(48, 8, i) for i in (1, 2)]
    N, M, F = encs[0].N, encs[0].M, 600
    rng = np.random.default_rng(7)
    d = to_dev(rng.standard_normal((F, M)) + 1j * rng.standard_normal((F, M)), np.complex64)
    p1 = build(P, ctx, encs[0], P.FP32, P.FLAG_UNCACHED)
    want = torch.empty((F, N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p1, d, want, refine_steps=1)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    xs = [torch.zeros((F, N), dtype=torch.complex64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    for x in xs:
        P.pinv_apply(ctx, p1, d, x, refine_steps=1, stream=side)
    P.pinv_plan_release(p1)
    p2 = P.pinv_build(ctx, encs[1], 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP32, P.FLAG_UNCACHED)
    y = torch.empty((F, N), dtype=torch.complex64, device="cuda")
    P.pinv_apply(ctx, p2, d, y)
    torch.cuda.synchronize()
    P.pinv_plan_wait(p2)
    P.pinv_plan_release(p2)
    for x in xs:
        assert torch.equal(x, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_paths_match_oracle(P, ctx, prec):
    """Applies of at most 8 frames stream R row by row; more frames run as MFMA
    tiles (ragged against 128-frame tiles here).  Both against the oracle's
    images, at the R path's tolerances, on 1, 3, 8, 9 and 150 frames."""
    o = oracle_case("ragged_c3")
    w, N, M = o["w"], o["w"].enc.N, o["w"].enc.M
    rng = np.random.default_rng(31)
    Fmax = 150
    d = rng.standard_normal((Fmax, M)) + 1j * rng.standard_normal((Fmax, M))
    x_ref = d @ o["R"].T          # the oracle's R applied frame by frame
    pr, cdt = (P.FP64, np.complex128) if prec == "fp64" else (P.FP32, np.complex64)
    plan = build(P, ctx, w.enc, pr, flags=P.FLAG_UNCACHED)
    try:
        for F in (1, 3, 8, 9, Fmax):
            dd = to_dev(d[:F], cdt)
            x = torch.full((F, N), float("nan"), dtype=dd.dtype, device="cuda")
            torch.cuda.synchronize()
            P.pinv_apply(ctx, plan, dd, x)
            torch.cuda.synchronize()
            err = frame_rel(x.cpu().numpy().astype(np.complex128), x_ref[:F])
            tol = 1e-9 if prec == "fp64" else o["kappa"] * 1e-6
            print(f"{prec} F={F}: max err {err.max():.2e}")
            assert err.max() < tol, (F, err.max())
    finally:
        P.pinv_plan_release(plan)


@pytest.mark.parametrize("prec,name,cprod", [
    ("fp64", "long_c4", "3m"), ("fp32", "long_c4", "3m"), ("fp32", "long_c4", "4m"),
    ("fp32", "long_odd", "3m"), ("fp32", "long_odd", "4m"), ("bf16x3", "long_c4", "auto")])
def test_few_frame_slices_match_oracle(P, ctx, prec, name, cprod):
    """Applies of a few frames stream R: row by row on the VALU (FP64 plans
    up to 8 frames, FP32 and BF16X3 plans up to 2), and 3 to 32 frames of
    FP32 and BF16X3 plans into the matrix cores.  With M >= 8192 the
    contraction is cut into slices (one per XCD for the row kernel, at most
    4096 columns for the streamed one), partials added in slice order.
    long_c4: M = 10400 (N = 480, ragged against the 128-row blocks); long_odd:
    M = 9003, odd (8-byte loads, a partial last chunk).  Against the oracle's R
    applied in FP64 at the R path's tolerances; BF16X3 plans also against
    their own R (copied out exactly) within 1e-5.  Both complex-product forms
    (the streamed kernel follows the plan's)."""
    o = oracle_case(name)
    w, N, M = o["w"], o["w"].enc.N, o["w"].enc.M
    assert M >= 8192
    rng = np.random.default_rng(41)
    d = rng.standard_normal((32, M)) + 1j * rng.standard_normal((32, M))
    pr, cdt = {"fp64": (P.FP64, np.complex128), "fp32": (P.FP32, np.complex64),
               "bf16x3": (P.BF16X3, np.complex64)}[prec]
    d = d.astype(cdt).astype(np.complex128)
    x_or = d @ o["R"].T
    form = {"3m": P.CPROD_3M, "4m": P.CPROD_4M, "auto": P.CPROD_AUTO}[cprod]
    plan = build(P, ctx, w.enc, pr, flags=P.FLAG_UNCACHED, cprod=form)
    try:
        x_own = None
        if prec == "bf16x3":
            R = torch.full((N, M), float("nan"), dtype=torch.complex64, device="cuda")
            P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
            torch.cuda.synchronize()
            x_own = d @ R.cpu().numpy().astype(np.complex128).T
        for F in (1, 2, 3, 4, 5, 8, 9, 12, 16, 17, 24, 32):
            dd = to_dev(d[:F], cdt)
            x = torch.full((F, N), float("nan"), dtype=dd.dtype, device="cuda")
            torch.cuda.synchronize()
            P.pinv_apply(ctx, plan, dd, x)
            torch.cuda.synchronize()
            xg = x.cpu().numpy().astype(np.complex128)
            err = frame_rel(xg, x_or[:F]).max()
            tol = {"fp64": 1e-9, "fp32": o["kappa"] * 1e-6, "bf16x3": o["kappa"] * 1e-4}[prec]
            print(f"{prec} {name} {cprod} F={F}: vs oracle R {err:.2e}")
            assert err < tol, (F, err)
            if x_own is not None:
                e_own = frame_rel(xg, x_own[:F]).max()
                assert e_own < 1e-5, (F, e_own)
    finally:
        P.pinv_plan_release(plan)


@pytest.mark.parametrize("prec,cprod", [("fp64", "auto"), ("fp32", "3m"), ("fp32", "4m"),
                                        ("bf16x3", "auto")])
@pytest.mark.parametrize("shape", ["16x18", "15x17"])
def test_few_frame_tiny_shapes_match_oracle(P, ctx, prec, cprod, shape):
    """Applies (Eq. 3) at tiny shapes, where the few-frame kernels run one
    workgroup with waves past N and fewer than 32 columns: N = 16, M = 18 (the
    streamed kernel's partial chunk alone) and N = 15, M = 17 (odd M: 8-byte
    loads; split-packed rows padded to 32).  Every path: rows, streamed
    (16- and 32-frame blocks) and tiles (33 frames).  Against the oracle's R
    applied in FP64 at the R path's tolerances."""
    nx, ny, C, K = {"16x18": (4, 4, 2, 9), "15x17": (5, 3, 1, 17)}[shape]
    w = synth.small_case(seed=107, nx=nx, ny=ny, C=C, K=K, F=1)
    enc = w.enc
    N, M = enc.N, enc.M
    assert M >= N and M < 32
    ob = oracle.Build(enc, rel=1e-3)
    R_or = ob.recon_matrix()
    ev = np.linalg.eigvalsh(ob.G + ob.lam * np.eye(N))
    kappa = ev[-1] / ev[0]
    rng = np.random.default_rng(43)
    d = rng.standard_normal((33, M)) + 1j * rng.standard_normal((33, M))
    pr, cdt = {"fp64": (P.FP64, np.complex128), "fp32": (P.FP32, np.complex64),
               "bf16x3": (P.BF16X3, np.complex64)}[prec]
    d = d.astype(cdt).astype(np.complex128)
    form = {"3m": P.CPROD_3M, "4m": P.CPROD_4M, "auto": P.CPROD_AUTO}[cprod]
    plan = build(P, ctx, enc, pr, flags=P.FLAG_UNCACHED, cprod=form)
    try:
        for F in (1, 2, 3, 5, 16, 17, 32, 33):
            dd = to_dev(d[:F], cdt)
            x = torch.full((F, N), float("nan"), dtype=dd.dtype, device="cuda")
            torch.cuda.synchronize()
            P.pinv_apply(ctx, plan, dd, x)
            torch.cuda.synchronize()
            xg = x.cpu().numpy().astype(np.complex128)
            err = frame_rel(xg, d[:F] @ R_or.T).max()
            tol = {"fp64": 1e-9, "fp32": kappa * 1e-6, "bf16x3": kappa * 1e-4}[prec]
            print(f"{prec} {cprod} {shape} F={F}: {err:.2e} (kappa {kappa:.2g})")
            assert err < tol, (F, err)
    finally:
        P.pinv_plan_release(plan)


def test_cache_hit_and_release(P, ctx):
    o = oracle_case("species_b0")
    a = build(P, ctx, o["w"].enc, P.FP32)
    b = P.pinv_build(ctx, o["w"].enc, 1e-3, P.LAMBDA_REL_MEAN_DIAG, P.FP32)
    assert a == b
    used, budget, n = P.pinv_context_usage(ctx)
    assert n >= 1 and used <= budget
    P.pinv_plan_release(a)
    P.pinv_plan_release(b)
    freed = P.pinv_cache_trim(ctx)
    assert freed > 0


@pytest.mark.parametrize("cprod", ["3m", "4m"])
@pytest.mark.parametrize("nb", [64, 128])
@pytest.mark.parametrize("name", ["ragged_c3", "species_b0"])
def test_factorisation_forms_match_oracle(P, ctx, name, nb, cprod):
    """The blocked factorisation with L^-1 alongside (Eq. 6, Eq. 8; Sec. 2.3)
    updating the trailing matrix every 64 columns or every 128 (two-level),
    under either product form of the plan's W and R: L^-1 element by element
    within 1e-9 of the oracle's forward substitution, R likewise.  ragged_c3:
    N = 480, 7.5 blocks (the last pair ragged); species_b0: N = 288, 4.5 blocks
    (a single step after two pairs)."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    form = P.CPROD_3M if cprod == "3m" else P.CPROD_4M
    plan = build(P, ctx, enc, P.FP64, flags=P.FLAG_UNCACHED, cprod=form, nb=nb)
    try:
        Li = torch.empty((N, N), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_LINV, Li)
        R = torch.empty((N, M), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    Li = Li.cpu().numpy()
    assert np.max(np.abs(np.triu(Li, 1))) == 0.0   # lower triangular
    assert max_rel_entry(np.tril(Li), o["Linv"]) < 1e-9
    assert max_rel_entry(R.cpu().numpy(), o["R"]) < 1e-9


@pytest.mark.parametrize("cprod", ["3m", "4m"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["ragged_c3", "aligned_species_b0"])
def test_product_forms_match_oracle(P, ctx, name, prec, cprod):
    """W, R and the apply with three real products per complex product (Gauss)
    or four.  FP64 plans: R element by element and the images within 1e-9 of
    the oracle either way.  FP32 plans: images within kappa * 1e-6 unrefined
    and 1e-5 after two refinement steps."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    form = P.CPROD_3M if cprod == "3m" else P.CPROD_4M
    pr, cdt = (P.FP64, np.complex128) if prec == "fp64" else (P.FP32, np.complex64)
    plan = build(P, ctx, enc, pr, flags=P.FLAG_UNCACHED, cprod=form)
    try:
        assert P.pinv_plan_info_get(plan)["cprod"] == form
        d = to_dev(o["d"], cdt)
        x0 = torch.empty((d.shape[0], N), dtype=d.dtype, device="cuda")
        x2 = torch.empty_like(x0)
        P.pinv_apply(ctx, plan, d, x0)
        P.pinv_apply(ctx, plan, d, x2, refine_steps=2)
        # 150 frames: the MFMA apply tiles (the 5 frames above stream R row by row)
        rng = np.random.default_rng(77)
        dm = rng.standard_normal((150, M)) + 1j * rng.standard_normal((150, M))
        xm = torch.empty((150, N), dtype=d.dtype, device="cuda")
        P.pinv_apply(ctx, plan, to_dev(dm, cdt), xm)
        R = torch.empty((N, M), dtype=d.dtype, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    e0 = frame_rel(x0.cpu().numpy().astype(np.complex128), o["x"]).max()
    e2 = frame_rel(x2.cpu().numpy().astype(np.complex128), o["x"]).max()
    em = frame_rel(xm.cpu().numpy().astype(np.complex128), dm @ o["R"].T).max()
    print(f"{name} {prec} {cprod}: err0 {e0:.2e} err2 {e2:.2e} mfma-apply {em:.2e}")
    if prec == "fp64":
        assert max_rel_entry(R.cpu().numpy(), o["R"]) < 1e-9
        assert e0 < 1e-9 and e2 < 1e-9 and em < 1e-9
    else:
        assert e0 < o["kappa"] * 1e-6 and em < o["kappa"] * 1e-6
        assert e2 < 1e-5


@pytest.mark.parametrize("form", ["psf", "shared", "full"])
@pytest.mark.parametrize("name", ["ragged_c3", "aligned_c2"])
def test_gram_forms_match_oracle(P, ctx, name, form):
    """The Gram through the point-spread function (offset grid times coil
    cross-products), on MFMA over one coil's samples times the coil
    cross-products, or over all M rows: FP64 plans, element by element within
    1e-12 of max|G|, and the same images (1e-9)."""
    o = oracle_case(name)
    enc, N = o["w"].enc, o["w"].enc.N
    g = {"psf": P.GRAM_PSF, "shared": P.GRAM_SHARED, "full": P.GRAM_FULL}[form]
    plan = build(P, ctx, enc, P.FP64, flags=P.FLAG_UNCACHED, gram=g)
    try:
        assert P.pinv_plan_info_get(plan)["gram_form"] == g
        G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
        d = to_dev(o["d"], np.complex128)
        x = torch.empty((d.shape[0], N), dtype=d.dtype, device="cuda")
        P.pinv_apply(ctx, plan, d, x)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    G = G.cpu().numpy()
    # the kept Gram is full Hermitian: both triangles against the oracle
    assert np.max(np.abs(G - o["b"].G)) <= 1e-12 * np.max(np.abs(o["b"].G))
    assert frame_rel(x.cpu().numpy(), o["x"]).max() < 1e-9


def test_psf_gram_with_species(P, ctx):
    """Species without an off-resonance map keep the offset structure (one PSF
    per species pair): the PSF Gram of a two-species encoding against the
    oracle, element by element."""
    w = synth.small_case(seed=151, nx=14, ny=11, C=3, K=640, F=2, species=[0.0, 210.0])
    enc, N = w.enc, w.enc.N
    Go = oracle.gram(enc)
    plan = build(P, ctx, enc, P.FP64, flags=P.FLAG_UNCACHED)
    try:
        assert P.pinv_plan_info_get(plan)["gram_form"] == P.GRAM_PSF
        G = torch.empty((N, N), dtype=torch.complex128, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_GRAM, G)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    assert np.max(np.abs(G.cpu().numpy() - Go)) <= 1e-12 * np.max(np.abs(Go))


@pytest.mark.parametrize("name", list(CASES))
def test_r_formed_in_fp64_matches_oracle(P, ctx, name):
    """FP32 plans with PINV_FLAG_R_FP64: W and R formed in FP64 and R rounded
    once to complex64.  R within the one rounding (2^-24 of each entry, so
    2^-23 of max|R| with room for the FP64 products) of the oracle's, element
    by element; unrefined FP32 applies within 1e-5 of the oracle's images
    (row-streaming and MFMA paths), where plain FP32 plans need refinement."""
    o = oracle_case(name)
    enc, N, M = o["w"].enc, o["w"].enc.N, o["w"].enc.M
    plan = build(P, ctx, enc, P.FP32, flags=P.FLAG_UNCACHED | P.FLAG_R_FP64)
    try:
        info = P.pinv_plan_info_get(plan)
        assert info["r_fp64"] and info["prec"] == P.FP32
        R = torch.empty((N, M), dtype=torch.complex64, device="cuda")
        P.pinv_plan_copy_buffer(plan, P.BUF_R, R)
        d = to_dev(o["d"], np.complex64)
        x = torch.empty((d.shape[0], N), dtype=torch.complex64, device="cuda")
        P.pinv_apply(ctx, plan, d, x)
        d40 = to_dev(np.tile(o["d"], (14, 1))[:40], np.complex64)
        x40 = torch.empty((40, N), dtype=torch.complex64, device="cuda")
        P.pinv_apply(ctx, plan, d40, x40)
        torch.cuda.synchronize()
    finally:
        P.pinv_plan_release(plan)
    eR = max_rel_entry(R.cpu().numpy().astype(np.complex128), o["R"])
    e = frame_rel(x.cpu().numpy().astype(np.complex128), o["x"]).max()
    e40 = frame_rel(x40.cpu().numpy().astype(np.complex128), np.tile(o["x"], (14, 1))[:40]).max()
    print(f"{name}: R entry err {eR:.2e} image err {e:.2e} / {e40:.2e} (kappa {o['kappa']:.3g})")
    assert eR <= 2.0 ** -23
    assert e < 1e-5 and e40 < 1e-5
