"""Seeded synthetic inputs for Randomly Pivoted LU (RPLU) runs.

This module builds matrices, Cauchy-like generators and job mixes. It holds
none of the method's arithmetic (no masses, sampling, pivoting or Schur
updates); both the CPU oracle and the HIP path take their inputs from here.

Inputs follow the shapes and spectra of the paper's workloads:

* dense test matrices A = U diag(sigma) V^T with orthonormal U, V and a chosen
  singular-value decay (the synthetic matrices of Sec. 3, Fig. 3: sigma_k
  proportional to 1/k^2 or rho^k);
* Cauchy matrices A_ij = 1/(x_i - y_j) on two interleaved spirals against a
  clustered set with outliers (the geometry of the spiral example of Fig. 1);
* Cauchy-like generators (eq. cauchy-like) and Loewner generators with the
  alpha scaling (eq. loewner-generators, Sec. 5.2).

The paper prints no coordinates for Fig. 1; the spiral/cluster parameters
below are a stated stand-in, not the paper's data.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "haar_orthonormal", "dense_with_spectrum", "config1_dense_512",
    "random_dense", "rank_r_dense", "spiral_cluster_points",
    "config2_cauchy_spirals", "cauchy_like_random", "loewner_generators",
    "batched_instance_specs", "batched_instance", "serving_arrivals",
    "dense_reflector_matrix_device",
]


# ---------------------------------------------------------------- dense inputs

def haar_orthonormal(rng: np.random.Generator, n: int, r: int,
                     complex_: bool = False) -> np.ndarray:
    """n x r matrix with orthonormal columns: Q of a Gaussian's QR, with the
    column signs fixed by sign(diag R) so that Q is Haar distributed."""
    if complex_:
        Z = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
    else:
        Z = rng.standard_normal((n, r))
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    ph = d / np.where(np.abs(d) == 0, 1.0, np.abs(d))
    return Q * ph[None, :]


def dense_with_spectrum(n: int, m: int, sigma: np.ndarray, seed,
                        complex_: bool = False) -> np.ndarray:
    """A = U diag(sigma) V^* with U (n x r), V (m x r) Haar orthonormal,
    r = len(sigma) <= min(n, m). U is drawn first, V second."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    assert r <= min(n, m)
    rng = np.random.default_rng(seed)
    U = haar_orthonormal(rng, n, r, complex_)
    V = haar_orthonormal(rng, m, r, complex_)
    return (U * sigma[None, :]) @ V.conj().T


def config1_dense_512(seed: int = 0) -> np.ndarray:
    """Dense FP64 512 x 512, sigma_i = 0.8^i (i = 1..512), Haar U and V."""
    n = 512
    sigma = 0.8 ** np.arange(1, n + 1, dtype=np.float64)
    return dense_with_spectrum(n, n, sigma, seed)


def random_dense(n: int, m: int, seed, complex_: bool = False) -> np.ndarray:
    """i.i.d. standard Gaussian entries (complex: independent re and im)."""
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    return rng.standard_normal((n, m))


def rank_r_dense(n: int, m: int, r: int, seed, complex_: bool = False) -> np.ndarray:
    """Exactly rank-r (in exact arithmetic) product X Y^T of Gaussians."""
    rng = np.random.default_rng(seed)
    if complex_:
        X = rng.standard_normal((n, r)) + 1j * rng.standard_normal((n, r))
        Y = rng.standard_normal((r, m)) + 1j * rng.standard_normal((r, m))
    else:
        X = rng.standard_normal((n, r))
        Y = rng.standard_normal((r, m))
    return X @ Y


def _compact_wy(Wm: np.ndarray) -> np.ndarray:
    """T of the compact WY form H_1 H_2 ... H_q = I - W T W^T of the
    reflectors H_l = I - tau_l w_l w_l^T, tau_l = 2 / (w_l^T w_l) (T upper
    triangular, built column by column)."""
    q = Wm.shape[1]
    tau = 2.0 / np.sum(Wm * Wm, axis=0)
    gram = Wm.T @ Wm
    T = np.zeros((q, q))
    for j in range(q):
        T[j, j] = tau[j]
        if j:
            T[:j, j] = -tau[j] * (T[:j, :j] @ gram[:j, j])
    return T


def dense_reflector_matrix_device(n: int, sigma_power: float = -2.0, q: int = 256,
                                  seed: int = 3, device="cuda:0", dtype=None):
    """Large square test matrix A = U diag(sigma) V^T, sigma_i = i^sigma_power,
    built on `device` with torch (FP64, then cast to dtype). U and V are
    exactly orthogonal products of q seeded full-support Householder
    reflectors, applied in compact WY form with three GEMMs per side, so no
    n x n QR is needed. (With q << n the singular vectors stay close to the
    coordinate axes; the spectrum is exact.)"""
    import torch
    rng = np.random.default_rng(seed)
    Wu = rng.standard_normal((n, q))
    Wv = rng.standard_normal((n, q))
    Tu, Tv = _compact_wy(Wu), _compact_wy(Wv)
    f64 = torch.float64
    sig = torch.arange(1, n + 1, dtype=f64, device=device) ** sigma_power
    Wu_d = torch.from_numpy(Wu).to(device)
    Wv_d = torch.from_numpy(Wv).to(device)
    Tu_d = torch.from_numpy(Tu).to(device)
    Tv_d = torch.from_numpy(Tv).to(device)
    # U diag(sigma) = diag(sigma) - Wu (Tu (Wu^T diag(sigma)))
    R = (Tu_d @ (Wu_d.T.contiguous() * sig[None, :])).contiguous()
    M = -(Wu_d @ R)
    del R
    M.diagonal().add_(sig)
    # A = M V^T with V^T = I - Wv Tv^T Wv^T
    P = (M @ Wv_d).contiguous()
    Q = (Tv_d.T.contiguous() @ Wv_d.T.contiguous()).contiguous()
    M -= P @ Q
    del P, Q
    if dtype is not None and dtype != f64:
        out = M.to(dtype)
        del M
        return out
    return M


# --------------------------------------------------------------- Cauchy inputs

def spiral_cluster_points(n: int = 20000, m: int = 20000, seed: int = 2,
                          outlier_frac: float = 0.05):
    """x: two interleaved spirals (radius 1..3, four turns), n points;
    y: a Gaussian cluster at 5+0i (sd 0.3 per coordinate) plus a fraction of
    outliers uniform in the disk |y - 5| <= 1.5, m points."""
    half = (n + 1) // 2
    tau = np.linspace(0.0, 1.0, half)
    x = np.empty(n, dtype=np.complex128)
    for s in (0, 1):
        pts = (1.0 + 2.0 * tau) * np.exp(1j * (8.0 * np.pi * tau + s * np.pi))
        x[s::2] = pts[: len(x[s::2])]
    rng = np.random.default_rng(seed)
    n_out = int(round(outlier_frac * m))
    n_cl = m - n_out
    z = rng.standard_normal((n_cl, 2))
    cluster = 5.0 + 0.3 * (z[:, 0] + 1j * z[:, 1])
    rad = 1.5 * np.sqrt(rng.random(n_out))
    ang = 2.0 * np.pi * rng.random(n_out)
    outl = 5.0 + rad * np.exp(1j * ang)
    y = np.concatenate([cluster, outl]).astype(np.complex128)
    return x, y


def config2_cauchy_spirals(n: int = 20000, m: int = 20000, seed: int = 2):
    """Cauchy matrix A_ij = 1/(x_i - y_j) as displacement-rank-1 generators
    G = ones(n,1), B = ones(1,m) over the spiral/cluster geometry."""
    x, y = spiral_cluster_points(n, m, seed)
    G = np.ones((n, 1), dtype=np.complex128)
    B = np.ones((1, m), dtype=np.complex128)
    return x, y, G, B


def cauchy_like_random(n: int, m: int, p: int, seed, separated: bool = True):
    """Random Cauchy-like generators (eq. cauchy-like): x in the unit disk,
    y in the annulus 2 <= |y| <= 3 (well separated), G and B complex
    Gaussian (n x p and p x m)."""
    rng = np.random.default_rng(seed)
    rx = np.sqrt(rng.random(n))
    x = rx * np.exp(2j * np.pi * rng.random(n))
    if separated:
        ry = np.sqrt(4.0 + 5.0 * rng.random(m))   # uniform in area on [2,3]
    else:
        ry = 1.2 + rng.random(m)
    y = ry * np.exp(2j * np.pi * rng.random(m))
    G = (rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))) / math.sqrt(2)
    B = (rng.standard_normal((p, m)) + 1j * rng.standard_normal((p, m))) / math.sqrt(2)
    return x.astype(np.complex128), y.astype(np.complex128), G, B


def loewner_generators(fx: np.ndarray, fy: np.ndarray):
    """Generators of the Loewner matrix (f^x_i - f^y_j)/(x_i - y_j)
    (eq. loewner-generators): G = [f^x/alpha, alpha], B = [alpha; -f^y/alpha],
    alpha = sqrt(max(max|f^x|, max|f^y|))."""
    fx = np.asarray(fx, dtype=np.complex128)
    fy = np.asarray(fy, dtype=np.complex128)
    alpha = math.sqrt(max(np.max(np.abs(fx)), np.max(np.abs(fy))))
    G = np.stack([fx / alpha, np.full_like(fx, alpha)], axis=1)
    B = np.stack([np.full_like(fy, alpha), -fy / alpha], axis=0)
    return G, B


# ------------------------------------------------------------ batched / serve

@dataclass
class InstanceSpec:
    index: int
    n: int
    m: int
    r: float          # geometric decay rate: sigma_i = r^i


def batched_instance_specs(count: int = 4096, seed: int = 4,
                           lo: int = 64, hi: int = 1024):
    """Shapes and decay rates of the batched workload: n, m ~ U{lo..hi}
    independently, r ~ U[0.5, 0.95]."""
    rng = np.random.default_rng(seed)
    n = rng.integers(lo, hi + 1, size=count)
    m = rng.integers(lo, hi + 1, size=count)
    r = rng.uniform(0.5, 0.95, size=count)
    return [InstanceSpec(b, int(n[b]), int(m[b]), float(r[b])) for b in range(count)]


def batched_instance(spec: InstanceSpec, seed: int = 4) -> np.ndarray:
    """A = U diag(r^i) V^T (i = 1..min(n,m)) for one batched instance, with
    its own seed [seed, index]."""
    k = min(spec.n, spec.m)
    sigma = spec.r ** np.arange(1, k + 1, dtype=np.float64)
    return dense_with_spectrum(spec.n, spec.m, sigma, [seed, spec.index])


def _stiefel_batched_device(rows_k, seeds, device):
    """Orthonormal factors Q (rows x k) of Gaussians, for many shapes at once.

    Each Gaussian G (rows x k, from torch's device generator seeded by its
    seed) has the unique QR factorisation G = Q R with diag(R) > 0; Q is
    computed by CholeskyQR2 (R1 = chol(G^T G), Q1 = G R1^-1, then the same on
    Q1), which yields that Q. Shapes are grouped into buckets of rows and k
    rounded up to 128 and processed as batches: G is zero-padded, and the
    padded diagonal block of each Gram matrix is set to the identity, so the
    Cholesky factor and the solve act on the true block alone. A bucket whose
    Cholesky fails (a nearly rank-deficient draw) falls back to Householder
    QR per matrix."""
    import torch
    f64 = torch.float64
    out = [None] * len(rows_k)
    buckets = {}
    for q, (r, k) in enumerate(rows_k):
        key = ((r + 127) // 128 * 128, (k + 127) // 128 * 128)
        buckets.setdefault(key, []).append(q)
    g = torch.Generator(device=device)
    for (R, K), idx in sorted(buckets.items()):
        for c0 in range(0, len(idx), 64):
            part = idx[c0:c0 + 64]
            Gp = torch.zeros((len(part), R, K), dtype=f64, device=device)
            pad = torch.zeros((len(part), K), dtype=f64, device=device)
            for b, q in enumerate(part):
                r, k = rows_k[q]
                g.manual_seed(seeds[q])
                Gp[b, :r, :k] = torch.randn((r, k), generator=g, device=device, dtype=f64)
                pad[b, k:] = 1.0
            Q = Gp
            ok = True
            for _ in range(2):
                Gram = Q.transpose(1, 2).contiguous() @ Q
                Gram += torch.diag_embed(pad)
                L, info = torch.linalg.cholesky_ex(Gram)
                if int(info.abs().sum()) != 0:
                    ok = False
                    break
                # Q <- Q L^-T  (L^T = R, upper triangular)
                Q = torch.linalg.solve_triangular(L.transpose(1, 2).contiguous(), Q, upper=True,
                                                  left=False)
            for b, q in enumerate(part):
                r, k = rows_k[q]
                if ok:
                    out[q] = Q[b, :r, :k].contiguous()
                else:
                    g.manual_seed(seeds[q])
                    G = torch.randn((r, k), generator=g, device=device, dtype=f64)
                    Qh, Rh = torch.linalg.qr(G)
                    out[q] = Qh * torch.sign(torch.diagonal(Rh))[None, :]
    return out


def batched_instances_device(specs, seed: int = 4, device="cuda:0", dtype=None):
    """The batched workload built on `device` (torch): for each spec,
    A = U diag(r^i) V^T (i = 1..min(n, m)) with U, V the orthonormal Q
    factors (diag(R) > 0) of Gaussians drawn from torch's device generator,
    seeded with seed * 2^32 + 2 * index (U) and + 1 (V). Returns a list of
    tensors of `dtype` (default float32)."""
    import torch
    dtype = dtype or torch.float32
    shapes, seeds = [], []
    for sp in specs:
        k = min(sp.n, sp.m)
        shapes += [(sp.n, k), (sp.m, k)]
        seeds += [seed * (1 << 32) + 2 * sp.index, seed * (1 << 32) + 2 * sp.index + 1]
    Q = _stiefel_batched_device(shapes, seeds, device)
    out = []
    for q, sp in enumerate(specs):
        k = min(sp.n, sp.m)
        U, V = Q[2 * q], Q[2 * q + 1]
        sig = sp.r ** torch.arange(1, k + 1, device=device, dtype=torch.float64)
        A = (U * sig[None, :]) @ V.T.contiguous()
        out.append(A.to(dtype).contiguous())
        Q[2 * q] = Q[2 * q + 1] = None
    return out


@dataclass
class Arrival:
    t: float                  # arrival time (s)
    kind: str                 # "dense" | "cauchy"
    n: int
    stream: int
    extra: dict = field(default_factory=dict)


def serving_arrivals(rate: float = 200.0, duration: float = 60.0, seed: int = 5,
                     dense_frac: float = 0.7, dense_n=(256, 8192),
                     cauchy_n=(10_000, 100_000)):
    """Poisson arrivals: exponential inter-arrival times at `rate` per
    second; each job is dense (probability dense_frac, square n ~ U{dense_n})
    or Cauchy-like (square n ~ U{cauchy_n})."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if rng.random() < dense_frac:
            n = int(rng.integers(dense_n[0], dense_n[1] + 1))
            out.append(Arrival(t, "dense", n, k))
        else:
            n = int(rng.integers(cauchy_n[0], cauchy_n[1] + 1))
            out.append(Arrival(t, "cauchy", n, k))
        k += 1
    return out


def serving_dense_pool(count: int = 64, n_range=(256, 8192), decay: float = 0.9, seed: int = 5,
                       rank_cut: int = 320, device="cuda:0", dtype=None):
    """The dense inputs of the serving workload: `count` square matrices with
    n ~ U{n_range} (numpy default_rng(seed + 1)), A = U diag(decay^i) V^T with
    U, V the orthonormal Q factors of device Gaussians. Singular values past
    rank_cut (decay^320 ~ 2e-15 for 0.9) are below single precision relative
    to sigma_1 and are left out. Returns (list of n, list of tensors)."""
    import torch
    dtype = dtype or torch.float32
    rng = np.random.default_rng(seed + 1)
    ns = [int(v) for v in rng.integers(n_range[0], n_range[1] + 1, size=count)]
    shapes, seeds = [], []
    for q, n in enumerate(ns):
        r = min(n, rank_cut)
        shapes += [(n, r), (n, r)]
        seeds += [(seed << 32) + 2 * q + 1_000_000, (seed << 32) + 2 * q + 1_000_001]
    Q = _stiefel_batched_device(shapes, seeds, device)
    out = []
    for q, n in enumerate(ns):
        r = min(n, rank_cut)
        sig = decay ** torch.arange(1, r + 1, device=device, dtype=torch.float64)
        A = (Q[2 * q] * sig[None, :]) @ Q[2 * q + 1].T.contiguous()
        out.append(A.to(dtype).contiguous())
        Q[2 * q] = Q[2 * q + 1] = None
    return ns, out


def serving_cauchy_pool(count: int = 32, n_range=(10_000, 100_000), seed: int = 5,
                        device="cuda:0"):
    """The Cauchy-like inputs of the serving workload: square n ~ U{n_range}
    (numpy default_rng(seed + 2)); x uniform in the unit disk, y uniform in
    the annulus 2 <= |y| <= 3, p = 1 with g, b ~ CN(0, 1) (a scaled Cauchy
    matrix), drawn on the device from torch's generator. Returns a list of
    (x, y, G, B) complex128 tensors."""
    import torch
    rng = np.random.default_rng(seed + 2)
    ns = [int(v) for v in rng.integers(n_range[0], n_range[1] + 1, size=count)]
    g = torch.Generator(device=device)
    out = []
    f64 = torch.float64
    for q, n in enumerate(ns):
        g.manual_seed((seed << 32) + 2_000_000 + q)
        u = torch.rand(4, n, generator=g, device=device, dtype=f64)
        x = torch.sqrt(u[0]) * torch.exp(2j * math.pi * u[1])
        y = torch.sqrt(4.0 + 5.0 * u[2]) * torch.exp(2j * math.pi * u[3])
        z = torch.randn(4, n, generator=g, device=device, dtype=f64) / math.sqrt(2.0)
        G = (z[0] + 1j * z[1]).reshape(n, 1).contiguous()
        B = (z[2] + 1j * z[3]).reshape(1, n).contiguous()
        out.append((x.contiguous(), y.contiguous(), G, B))
    return out
