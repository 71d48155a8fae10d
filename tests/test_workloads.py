"""The seeded input generator: field statistics, resolution independence, FP32 wrap."""
import numpy as np

import workloads as W


def test_displacement_rms_and_grid_matches_direct_sum():
    psi = W.displacement_grid(24, 6)
    assert abs(np.sqrt((psi ** 2).sum(0).mean()) - W.RMS_PSI) < 1e-12
    q = W.lattice_q(24)
    idx = np.random.default_rng(0).choice(24 ** 3, 40, replace=False)
    direct = W.displacement_at(q[idx], 6)
    grid = np.stack([psi[c].ravel()[idx] for c in range(3)], 1)
    np.testing.assert_allclose(grid, direct, rtol=0, atol=1e-15)


def test_same_field_on_two_resolutions():
    a = W.displacement_grid(16, 5)
    b = W.displacement_grid(32, 5)
    np.testing.assert_allclose(a, b[:, ::2, ::2, ::2], rtol=0, atol=1e-15)


def test_positions_are_wrapped_fp32_and_seeded():
    x, y, z = W.zeldovich(16, 5, 8.0)
    for c in (x, y, z):
        assert c.dtype == np.float32 and c.min() >= 0 and c.max() < 1
    x2, _, _ = W.zeldovich(16, 5, 8.0)
    assert np.array_equal(x, x2)
    x3, _, _ = W.zeldovich(16, 5, 8.0, seed=4)
    assert not np.array_equal(x, x3)


def test_rotations_are_orthonormal():
    R = W.random_rotations(16)
    np.testing.assert_allclose(R @ R.transpose(0, 2, 1), np.broadcast_to(np.eye(3), R.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-14)


def test_workload_table():
    assert W.TINY.tets == 196608 and W.MID.tets == 12582912 and W.STRESS.tets == 100663296
    assert len(W.BATCHED.growth) == 8 and W.BATCHED.n_views == 64
