"""Seeded input generators produce the stated spectra and geometry."""
import numpy as np
import torch

import workloads as W


def test_config1_spectrum():
    A = W.config1_dense_512()
    s = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, 0.8 ** np.arange(1, 513), rtol=1e-10, atol=1e-14)


def test_reflector_matrix_spectrum_cpu():
    A = W.dense_reflector_matrix_device(300, sigma_power=-2.0, q=40, seed=3, device="cpu")
    s = np.linalg.svd(A.numpy(), compute_uv=False)
    assert np.allclose(s, np.arange(1, 301) ** -2.0, rtol=1e-10, atol=1e-14)
    A32 = W.dense_reflector_matrix_device(64, q=8, device="cpu", dtype=torch.float32)
    assert A32.dtype == torch.float32


def test_spiral_cluster_geometry():
    x, y = W.spiral_cluster_points(2000, 2000, seed=2)
    assert np.all(np.abs(np.abs(x) - 2.0) <= 1.0 + 1e-12)          # radius 1..3
    assert np.min(np.abs(x[:, None] - y[None, :])) >= 0.1
    assert abs(np.median(y.real) - 5.0) < 0.1


def test_batched_specs():
    sp = W.batched_instance_specs(4096, seed=4)
    n = np.array([s.n for s in sp])
    r = np.array([s.r for s in sp])
    assert n.min() >= 64 and n.max() <= 1024 and 0.5 <= r.min() and r.max() <= 0.95
