"""The seeded generators: reproducible, in range, shaped like the workloads."""
import numpy as np
import pytest

from paper_2410_06129_amd import synth


def test_seeds_reproduce_bit_exactly():
    a, b = synth.radial_32x32_c1(), synth.radial_32x32_c1()
    assert np.array_equal(a.enc.k, b.enc.k)
    assert np.array_equal(a.images, b.images)
    assert np.array_equal(a.noise, b.noise)
    c1 = synth.coil_maps(16, 16, 4, synth.rng_for(2, 2))
    c2 = synth.coil_maps(16, 16, 4, synth.rng_for(2, 2))
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("traj,n", [("radial", 32), ("spiral", 64), ("spiral", 96)])
def test_trajectories_inside_band(traj, n):
    k = synth.golden_radial(n, 16, 128) if traj == "radial" else synth.vd_spiral(n, 4096)
    assert np.all(k >= -n / 2) and np.all(k < n / 2)


def test_workload_shapes():
    w1 = synth.radial_32x32_c1()
    assert (w1.enc.N, w1.enc.M) == (1024, 2048)
    w4 = synth.species5_32x32_c8(F=3)
    assert (w4.enc.N, w4.enc.M, w4.enc.S) == (5120, 49152, 5)
    assert np.max(np.abs(w4.enc.b0_hz)) == pytest.approx(30.0)
    assert w4.images.shape == (3, 5120)
    k = synth.vd_spiral(64, 4096)
    assert k.shape == (4096, 2)


def test_workloads_overdetermined():
    for n, C, K in [(32, 1, 2048), (64, 8, 4096), (96, 16, 8192), (32, 8, 6144)]:
        assert C * K >= 2 * n * n or (n == 32 and C == 8)


def test_dynamic_frames_bounded_change():
    x = synth.ellipse_phantom(16, 16, np.random.default_rng(1))
    f = synth.dynamic_frames(x, 20, np.random.default_rng(2))
    nz = np.abs(x) > 0
    ratio = np.abs(f[:, nz]) / np.abs(x[nz])[None, :]
    assert ratio.min() >= 0.95 - 1e-12 and ratio.max() <= 1.05 + 1e-12


def test_unit_noise_power():
    n = synth.unit_complex_noise((200000,), np.random.default_rng(0))
    assert abs(np.mean(np.abs(n) ** 2) - 1.0) < 0.01


def test_serving_trace():
    tr = synth.serving_trace()
    assert 380 < len(tr) < 580
    assert all(50 <= r.frames <= 2000 for r in tr)
    assert tr[0].new_build
    frac_new = np.mean([r.new_build for r in tr])
    assert 0.2 < frac_new < 0.4
    arr = [r.arrival_s for r in tr]
    assert arr == sorted(arr) and arr[-1] <= 120.0
