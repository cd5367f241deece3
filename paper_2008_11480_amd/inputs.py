"""Seeded synthetic workloads for the SPD solver.

This module only *builds inputs*.  It contains none of the solver's arithmetic
(no scaling, no Newton-Schulz step, no Richardson update), so both the HIP path
and the CPU oracle may draw their inputs from it.

The paper's own simulation uses the Gram matrix of a harmonic regressor with
three frequencies (Section 7); its data set is not published, so the recipes
below stand in for it:

* ``spd_qlq``: ``A = Q diag(lam) Q^T`` with ``Q`` Haar-orthogonal (QR of a
  seeded Gaussian, column signs fixed by ``sign(diag R)``) and ``lam``
  log-uniform in ``[1, kappa]`` with both ends pinned, so that
  ``cond_2(A) = kappa`` exactly.  ``b ~ N(0, 1)``.  The eigen-decomposition is
  returned as well; the closed-form error laws of the method are stated in it.
* ``harmonic_gram``: the Gram matrix of a harmonic regressor
  ``phi(t) = [cos w_1 t, sin w_1 t, ..., cos w_m t, sin w_m t]`` sampled at
  ``t = 1..4N`` (``N = 2m``), plus a ``1e-6 I`` ridge, and ``b = sum_t phi y``
  with ``y = phi^T theta_true + N(0, 0.01)`` (Section 1 names harmonic
  regressors as the SPD source).
* ``harmonic_batch``: many such systems with ``m ~ U{8..128}``.
* ``serving_trace``: Poisson arrivals of SPD requests with log-uniform sizes
  and condition numbers.

All generators use numpy's PCG64 (``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class SPDSystem:
    """One SPD system ``A theta = b`` with its spectral data (when known)."""

    A: np.ndarray  # (N, N) float64, C-contiguous, symmetric
    b: np.ndarray  # (N,) float64
    lam: np.ndarray | None = None  # eigenvalues (known for spd_qlq)
    Q: np.ndarray | None = None  # eigenvectors, columns (known for spd_qlq)
    seed: int = 0
    kappa: float | None = None

    @property
    def n(self) -> int:
        return int(self.A.shape[0])


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian, signs fixed."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.ascontiguousarray(q * d[None, :])


def loguniform_spectrum(n: int, kappa: float, rng: np.random.Generator) -> np.ndarray:
    """``n`` eigenvalues log-uniform in ``[1, kappa]``, first = 1, last = kappa."""
    if n == 1:
        return np.array([1.0])
    lam = np.exp(rng.uniform(0.0, math.log(kappa), size=n))
    lam[0] = 1.0
    lam[-1] = float(kappa)
    return lam


def spd_qlq(n: int, kappa: float, seed: int, with_eig: bool = True) -> SPDSystem:
    """``A = Q diag(lam) Q^T`` (symmetrised), ``b ~ N(0,1)``; all from ``seed``."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    lam = loguniform_spectrum(n, kappa, rng)
    a = (q * lam[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    b = rng.standard_normal(n)
    return SPDSystem(A=np.ascontiguousarray(a), b=b,
                     lam=lam if with_eig else None, Q=q if with_eig else None,
                     seed=seed, kappa=float(kappa))


def spd_qlq_device(n: int, kappa: float, seed: int, device="cuda"):
    """The ``spd_qlq`` recipe with the QR and the product done by torch on
    ``device`` (for large N): the same PCG64 draws (Gaussian, spectrum, b) in
    the same order, Q sign-fixed by ``sign(diag R)``.  Q differs from
    ``spd_qlq``'s only by the QR implementation's rounding.  Returns torch
    tensors ``(A, b, lam, Q)`` on ``device`` (float64)."""
    import torch
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n))
    lam = loguniform_spectrum(n, kappa, rng)
    b = rng.standard_normal(n)
    zt = torch.from_numpy(z).to(device)
    q, r = torch.linalg.qr(zt)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    q = q * d[None, :]
    lt = torch.from_numpy(lam).to(device)
    a = (q * lt[None, :]) @ q.T.contiguous()
    a = 0.5 * (a + a.T)
    return a.contiguous(), torch.from_numpy(b).to(device), lt, q.contiguous()


def householder_factors(n: int, kappa: float, seed: int, reflectors: int = 4):
    """Host draws of a serving-size SPD system ``A = Q diag(lam) Q^T`` with
    ``Q = H_1 H_2 ... H_r`` a product of ``reflectors`` seeded Householder
    reflections: ``lam`` log-uniform in ``[1, kappa]`` with both ends pinned,
    the reflection vectors ``V`` (rows), ``b ~ N(0, 1)``.  O(n) numbers."""
    rng = np.random.default_rng(seed)
    lam = loguniform_spectrum(n, kappa, rng)
    vs = rng.standard_normal((reflectors, n))
    b = rng.standard_normal(n)
    return lam, vs, b


def _wy_core(lam: np.ndarray, vs: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """``Q diag(lam) Q^T = diag(lam) + Z C Z^T`` for ``Q = H_1 ... H_r``
    (``H_i = I - tau_i v_i v_i^T``, ``tau_i = 2 / v_i^T v_i``): the compact WY
    form ``Q = I - W T W^T`` (``W = [v_1 .. v_r]``, ``T`` upper triangular,
    accumulated one reflection at a time) gives ``Z = [W, diag(lam) W]`` and
    ``C = [[T M T^T, -T], [-T^T, 0]]`` with ``M = W^T diag(lam) W``."""
    w = np.ascontiguousarray(vs.T)                      # n x r
    r = w.shape[1]
    t = np.zeros((r, r))
    for j in range(r):
        tau = 2.0 / float(w[:, j] @ w[:, j])
        if j:
            t[:j, j] = -tau * (t[:j, :j] @ (w[:, :j].T @ w[:, j]))
        t[j, j] = tau
    u = lam[:, None] * w
    m = w.T @ u
    c = np.zeros((2 * r, 2 * r))
    tmt = t @ m @ t.T
    c[:r, :r] = 0.5 * (tmt + tmt.T)                     # symmetric to the bit
    c[:r, r:] = -t
    c[r:, :r] = -t.T
    return np.concatenate([w, u], axis=1), c


def householder_pack(lam: np.ndarray, vs: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One host array holding what the device needs to make the system of
    :func:`householder_factors`: ``[Z C (n x 2r) | Z (n x 2r) | lam | b |
    zeros (theta) | V (r x n)]`` (see :func:`_wy_core`)."""
    z, c = _wy_core(lam, vs)
    return np.concatenate([(z @ c).ravel(), z.ravel(), lam, b, np.zeros_like(b), vs.ravel()])


def householder_unpack_device(packed: np.ndarray, n: int, reflectors: int = 4, device="cuda"):
    """Device tensors ``(A, b, theta, lam, V)`` from :func:`householder_pack`:
    one upload, then ``A = (Z C) Z^T`` and ``diag(A) += lam`` (two device
    operations).  ``A`` is symmetric to the rounding of that product's
    summation order; ``theta`` is zero."""
    import torch
    w = 2 * reflectors
    dev = torch.from_numpy(packed).to(device)
    o = 0
    zc = dev[o:o + n * w].view(n, w)
    o += n * w
    z = dev[o:o + n * w].view(n, w)
    o += n * w
    lam = dev[o:o + n]
    b = dev[o + n:o + 2 * n]
    theta = dev[o + 2 * n:o + 3 * n]
    V = dev[o + 3 * n:].view(reflectors, n)
    a = zc @ z.T
    a.diagonal().add_(lam)
    return a, b, theta, lam, V


def householder_dense_pack(lam: np.ndarray, vs: np.ndarray, b: np.ndarray) -> np.ndarray:
    """``[A (n x n, row-major) | b | zeros (theta) | lam | V (r x n)]`` on the
    host, ``A = diag(lam) + (Z C) Z^T`` (for small systems, uploaded whole)."""
    z, c = _wy_core(lam, vs)
    a = (z @ c) @ z.T
    a[np.diag_indices_from(a)] += lam
    return np.concatenate([a.ravel(), b, np.zeros_like(b), lam, vs.ravel()])


def dense_unpack(dev, n: int, reflectors: int = 4):
    """Views ``(A, b, theta, lam, V)`` of a device copy of
    :func:`householder_dense_pack`'s array."""
    o = n * n
    return (dev[:o].view(n, n), dev[o:o + n], dev[o + n:o + 2 * n], dev[o + 2 * n:o + 3 * n],
            dev[o + 3 * n:o + 3 * n + reflectors * n].view(reflectors, n))


def spd_from_factors_device(lam: np.ndarray, vs: np.ndarray, b: np.ndarray, device="cuda"):
    """Device tensors ``(A, b, lam, V)`` (float64) of the system of
    :func:`householder_factors` (via :func:`householder_pack`)."""
    a, bt, _, lt, V = householder_unpack_device(householder_pack(lam, vs, b), lam.shape[0],
                                                vs.shape[0], device)
    return a, bt, lt, V


def spd_householder_device(n: int, kappa: float, seed: int, reflectors: int = 4,
                           device="cuda"):
    """Serving-size SPD system on ``device``: ``A = Q diag(lam) Q^T`` with ``Q``
    a product of ``reflectors`` seeded Householder reflections (O(n^2) work,
    so requests are cheap to make), ``lam`` log-uniform in ``[1, kappa]`` with
    both ends pinned, ``b ~ N(0, 1)``.  The method's convergence depends only
    on ``lam`` and ``alpha``.  Returns torch tensors ``(A, b, lam, V)``
    (float64); ``V`` holds the reflection vectors as rows, applied in order
    (``Q = H_1 H_2 ... H_r`` acting on ``diag(lam)``)."""
    lam, vs, b = householder_factors(n, kappa, seed, reflectors)
    return spd_from_factors_device(lam, vs, b, device)


def householder_solve_device(lam, V, b):
    """``A^{-1} b`` for a system from :func:`spd_householder_device`
    (``Q diag(1/lam) Q^T b`` with the same reflections): a closed form."""
    import torch
    x = b.clone()
    for i in range(V.shape[0]):            # Q^T b = H_r ... H_1 b
        v = V[i]
        x = x - (2.0 * torch.dot(v, x) / torch.dot(v, v)) * v
    x = x / lam
    for i in range(V.shape[0] - 1, -1, -1):   # Q y = H_1 ... H_r y
        v = V[i]
        x = x - (2.0 * torch.dot(v, x) / torch.dot(v, v)) * v
    return x


def spd_diag(lam: np.ndarray, seed: int) -> SPDSystem:
    """Diagonal SPD system with the given spectrum and ``b ~ N(0,1)``."""
    rng = np.random.default_rng(seed)
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.size
    return SPDSystem(A=np.diag(lam).copy(), b=rng.standard_normal(n), lam=lam.copy(),
                     Q=np.eye(n), seed=seed, kappa=float(lam.max() / lam.min()))


def spd_jacobi(n: int, seed: int, decades: float = 3.0, offdiag: float = 0.9) -> SPDSystem:
    """``A = D^(1/2) (I + E) D^(1/2)``: ``E`` symmetric with zero diagonal and
    every row sum of ``|E|`` equal to ``offdiag < 1`` (so ``I + E`` is strictly
    diagonally dominant and ``2 S - A`` is positive definite for
    ``S = diag(A) = D``, Section 2), ``D`` log-uniform over ``decades``
    decades.  The diagonal preconditioner sees the spectrum of ``I + E``; the
    scalar one sees that of ``A``.  ``b ~ N(0, 1)``."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n, n))
    e = 0.5 * (e + e.T)
    np.fill_diagonal(e, 0.0)
    if n > 1:
        rs = np.abs(e).sum(axis=1)
        e = e / np.sqrt(np.outer(rs, rs))        # symmetric scaling keeps E = E^T
        e *= offdiag / np.abs(e).sum(axis=1).max()
    d = 10.0 ** rng.uniform(0.0, decades, size=n)
    sq = np.sqrt(d)
    a = (np.eye(n) + e) * np.outer(sq, sq)
    a = 0.5 * (a + a.T)
    b = rng.standard_normal(n)
    return SPDSystem(A=np.ascontiguousarray(a), b=b, seed=seed)


def harmonic_gram(m: int, seed: int, ridge: float = 1e-6, noise_var: float = 0.01,
                  samples_per_dim: int = 4) -> SPDSystem:
    """Gram matrix of a harmonic regressor with ``m`` frequencies (``N = 2m``).

    ``phi(t)`` interleaves ``cos w_i t`` and ``sin w_i t``; ``t = 1..4N``;
    ``w_i ~ U(0, pi)``; ``theta_true ~ N(0, I)``; ``y = phi^T theta_true + e``
    with ``e ~ N(0, noise_var)``.
    """
    rng = np.random.default_rng(seed)
    n = 2 * m
    w = rng.uniform(0.0, math.pi, size=m)
    t = np.arange(1, samples_per_dim * n + 1, dtype=np.float64)
    phi = np.empty((t.size, n))
    phi[:, 0::2] = np.cos(np.outer(t, w))
    phi[:, 1::2] = np.sin(np.outer(t, w))
    theta_true = rng.standard_normal(n)
    y = phi @ theta_true + math.sqrt(noise_var) * rng.standard_normal(t.size)
    a = phi.T @ phi + ridge * np.eye(n)
    a = 0.5 * (a + a.T)
    b = phi.T @ y
    return SPDSystem(A=np.ascontiguousarray(a), b=b, seed=seed)


def harmonic_three(samples: int = 30, omegas=(0.40, 0.43, 0.47), seed: int = 6) -> SPDSystem:
    """Gram matrix of a harmonic regressor with three close frequencies
    (``N = 6``), the shape of the paper's comparison problem (Section 7):
    ``phi(t) = [cos w_i t, sin w_i t]_{i=1..3}``, ``t = 1..samples``,
    ``A = sum_t phi phi^T``, noise-free ``y = phi^T theta_true`` with
    ``theta_true ~ N(0, I)``, ``b = sum_t phi y``.  With the defaults
    kappa(A) ~ 4e3."""
    rng = np.random.default_rng(seed)
    t = np.arange(1, samples + 1, dtype=np.float64)
    phi = np.empty((t.size, 2 * len(omegas)))
    for i, w in enumerate(omegas):
        phi[:, 2 * i] = np.cos(w * t)
        phi[:, 2 * i + 1] = np.sin(w * t)
    theta_true = rng.standard_normal(phi.shape[1])
    a = phi.T @ phi
    a = 0.5 * (a + a.T)
    b = phi.T @ (phi @ theta_true)
    return SPDSystem(A=np.ascontiguousarray(a), b=b, seed=seed)


def harmonic_batch(count: int, seed: int, m_lo: int = 8, m_hi: int = 128) -> list[SPDSystem]:
    """``count`` harmonic Gram systems, ``m ~ U{m_lo..m_hi}``, per-system seeds
    spawned from ``seed``."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    children = ss.spawn(count)
    out = []
    for m, child in zip(ms, children):
        sub = int(child.generate_state(1)[0])
        out.append(harmonic_gram(int(m), sub))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    n: int
    kappa: float
    seed: int


def serving_trace(rate_per_s: float, duration_s: float, seed: int,
                  n_lo: int = 32, n_hi: int = 2048,
                  kappa_lo: float = 10.0, kappa_hi: float = 1e6) -> list[Request]:
    """Poisson arrivals; ``N = round(exp U(ln n_lo, ln n_hi))``,
    ``kappa = exp U(ln kappa_lo, ln kappa_hi)``, one seed per request."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        kappa = float(math.exp(rng.uniform(math.log(kappa_lo), math.log(kappa_hi))))
        out.append(Request(arrival_s=t, n=n, kappa=kappa, seed=int(rng.integers(0, 2**62))))
    return out


def random_symmetric_contraction(n: int, radius: float, seed: int) -> np.ndarray:
    """Random symmetric matrix with spectral radius ``radius`` (test operand)."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(n, rng)
    mu = rng.uniform(-radius, radius, size=n)
    mu[0] = radius
    f = (q * mu[None, :]) @ q.T
    return np.ascontiguousarray(0.5 * (f + f.T))


def shift_matrix(m: int) -> np.ndarray:
    """Nilpotent upper shift ``J`` (ones on the first super-diagonal).

    Powers of ``J`` are exact in floating point, so any polynomial in ``J``
    with small integer coefficients is evaluated exactly: this turns the
    matrix programs of the method into exact integer identities.
    """
    return np.eye(m, k=1)


# Workloads used by the tests and the benchmark, named by what they are.
WORKLOADS = {
    # N=64, kappa=100, order 4 squaring, 12 steps, target rel. residual 1e-13.
    "spd64_k1e2_o4": dict(n=64, kappa=1e2, seed=1, order=4, k_max=12, resid_tol=1e-13),
    # N=4096, kappa=1e4, order 8 squaring, to the ||F|| floor, FP64.
    "spd4096_k1e4_o8": dict(n=4096, kappa=1e4, seed=2, order=8, k_max=64, resid_tol=1e-12),
    # N=8192, kappa=1e6, composite (double) Newton-Schulz of order 8, mixed.
    "spd8192_k1e6_dns8": dict(n=8192, kappa=1e6, seed=3, order=8, k_max=64, resid_tol=1e-10),
}
