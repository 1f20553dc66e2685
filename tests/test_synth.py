"""Seeded input generator: determinism, geometry and statistics (no GPU)."""
import numpy as np

from paper_1807_08084_amd import synth


def test_deterministic_and_row_bands():
    a = synth.make_image(96, 80, 4, (2, 2), (1e-2, 1.0), 5)
    b = synth.make_image(96, 80, 4, (2, 2), (1e-2, 1.0), 5)
    assert np.array_equal(a.planes, b.planes)
    band = synth.make_image(96, 80, 4, (2, 2), (1e-2, 1.0), 5, rows=(17, 61))
    assert np.array_equal(band.planes, a.planes[:, 17:61])
    c = synth.make_image(96, 80, 4, (2, 2), (1e-2, 1.0), 6)
    assert not np.array_equal(a.planes, c.planes)


def test_chunking_independent_of_workers(monkeypatch):
    img = synth.make_image(700, 800, 3, (1, 1), (1e-8, 1.0), 2, per_pixel=True)
    monkeypatch.setattr(synth, "_workers", lambda: 1)
    img1 = synth.make_image(700, 800, 3, (1, 1), (1e-8, 1.0), 2, per_pixel=True)
    assert np.array_equal(img.planes, img1.planes)


def test_region_grid():
    img = synth.make_image(64, 96, 4, (2, 4), (1e-2, 1.0), 0)
    r = img.region_of
    assert r[0, 0] == 0 and r[0, 95] == 3 and r[63, 0] == 4 and r[63, 95] == 7
    assert r[31, 23] == 0 and r[32, 24] == 5
    assert np.bincount(r.ravel()).tolist() == [32 * 24] * 8


def test_hermitian_psd_and_unitary():
    rng = np.random.default_rng(3)
    U = synth.haar_unitary(rng, 1000)
    eye = np.einsum("mji,mjk->mik", np.conj(U), U)
    assert np.abs(eye - np.eye(3)).max() < 1e-14
    img = synth.workload_small()
    Z = synth.unpack(img.planes.reshape(9, -1))
    w = np.linalg.eigvalsh(Z)
    assert np.all(w[:, 0] > 0)  # N = 4 >= 3 looks: full rank


def test_mean_and_wishart_determinant_moment():
    """E[Z] = Sigma_c and E[det Z] = det(Sigma_c) N(N-1)(N-2)/N^3 (complex Wishart)."""
    for N in (3, 4, 8):
        img = synth.make_image(512, 512, N, (1, 1), (1e-1, 1.0), 40 + N)
        Z = synth.unpack(img.planes.reshape(9, -1))
        sig = img.sigma_regions[0]
        mean = Z.mean(axis=0)
        assert np.abs(mean - sig).max() <= 0.02 * np.abs(sig).max()
        det = np.linalg.det(Z).real
        want = np.linalg.det(sig).real * N * (N - 1) * (N - 2) / N ** 3
        assert abs(det.mean() / want - 1.0) < 0.03


def test_batch_recipe():
    shapes = synth.batch_shapes()
    px = [h * w for h, w, _ in shapes]
    assert len(shapes) == 64 and sum(px) == 77_940_374
    assert min(px) == 27_832 and max(px) == 9_938_360
    assert all(128 <= h <= 4096 and 128 <= w <= 4096 for h, w, _ in shapes)
    assert sorted({n for *_, n in shapes}) == [3, 4, 8, 16]


def test_wishart_sigma0():
    img = synth.make_image(8, 8, 8, (2, 2), (1e-2, 1.0), 3)
    z = img.planes.reshape(9, -1)
    s = synth.wishart_sigma0(z)
    tr = z[0] + z[1] + z[2]
    for k in range(3):
        assert np.allclose(s[k], z[k] + 0.1 * tr / 3)
    assert np.array_equal(s[3:], z[3:])


def test_paper_shaped_stand_ins():
    """M M^H with Re/Im(M) uniform on [-1, 1]: Hermitian positive definite,
    E[M M^H] = (2/3) 3 I = 2 I; chunks identical whatever the count; the
    450 x 600 image has the small recipe's planes at that shape."""
    p = synth.workload_paper_simulated(count=300000)
    z = synth.unpack(p)
    assert np.allclose(z, np.conj(np.transpose(z, (0, 2, 1))))
    assert np.all(np.linalg.eigvalsh(z[:20000]) > 0)
    mean = z.mean(axis=0)
    assert np.allclose(mean, 2.0 * np.eye(3), atol=0.02)
    q = synth.workload_paper_simulated(count=synth.CHUNK + 5)
    assert np.array_equal(q[:, :synth.CHUNK], p[:, :synth.CHUNK])
    a = synth.workload_airsar_standin()
    assert a.planes.shape == (9, 450, 600)
