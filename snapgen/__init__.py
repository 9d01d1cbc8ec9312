"""Seeded synthetic snapshot matrices (inputs only: no step of the method).

These stand in for the paper's datasets (Faces, V2D, CYF, YF), which are not
available: they keep the shape class (tall and thin, row mean-centred,
decaying or clustered spectra) of those workloads.  Both the oracle tests and
the GPU path consume the bytes produced here; nothing here computes any part
of the POD method.

All matrices are column-major (snapshot j is contiguous).  With torch the
storage is an (n, m) contiguous tensor ``At`` whose transpose is A; with
numpy an m x n Fortran-ordered array.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np


def _haar_columns(rng: np.random.Generator, m: int, k: int, project_out_ones: bool = False) -> np.ndarray:
    """First k columns of a Haar-distributed orthogonal matrix: QR of a
    Gaussian m x k matrix with the signs fixed so that diag(R) > 0.  With
    project_out_ones the Gaussian is first projected on the complement of
    the all-ones vector, so the columns are orthogonal to it."""
    G = rng.standard_normal((m, k))
    if project_out_ones:
        G = G - G.mean(axis=0, keepdims=True)
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def centre_rows_np(A: np.ndarray) -> np.ndarray:
    """Subtract each row's mean (accumulated in FP64), keeping the dtype."""
    mu = A.astype(np.float64).mean(axis=1, keepdims=True)
    return np.asfortranarray((A.astype(np.float64) - mu).astype(A.dtype))


@dataclass
class SpectrumMatrix:
    A: np.ndarray          # m x n, Fortran order
    U: np.ndarray          # m x q exact left factor of the noiseless part
    s: np.ndarray          # q prescribed singular values
    V: np.ndarray          # n x q exact right factor


def spectrum_matrix(m: int, n: int, s, noise_var: float, seed: int, centre: bool = True,
                    dtype=np.float64, v_orthogonal_to_ones: bool = True) -> SpectrumMatrix:
    """A = U diag(s) V^T + N(0, noise_var) with Haar U (m x q) and V (n x q).

    With ``v_orthogonal_to_ones`` V is Haar on the complement of the ones
    vector, so row centring leaves the noiseless part (and its exact
    singular values and subspaces) unchanged."""
    s = np.asarray(s, dtype=np.float64)
    q = s.shape[0]
    rng = np.random.default_rng(seed)
    U = _haar_columns(rng, m, q)
    V = _haar_columns(rng, n, q, project_out_ones=v_orthogonal_to_ones)
    A = (U * s[None, :]) @ V.T
    if noise_var > 0:
        A = A + math.sqrt(noise_var) * rng.standard_normal((m, n))
    A = np.asfortranarray(A.astype(dtype))
    if centre:
        A = centre_rows_np(A)
    return SpectrumMatrix(A, U, s, V)


def config_small_fp64(seed: int = 1001, m: int = 2000, n: int = 500) -> SpectrumMatrix:
    """Small FP64 workload: m x n, s_i = exp(-i/8) for i < 100 (0-based),
    Gaussian noise of variance 1e-8, rows centred."""
    q = min(100, m, n - 1)
    s = np.exp(-np.arange(q) / 8.0)
    return spectrum_matrix(m, n, s, 1e-8, seed, centre=True, dtype=np.float64)


def travelling_waves(m: int, n: int, n_modes: int, alpha: float, noise_var: float, seed: int,
                     centre: bool = True, device: str = "cpu", dtype=None, chunk: int = 256):
    """Sum of travelling waves a_j sin(kappa_j x - omega_j t + phi_j) on the
    grid x_i = i/m, t_j = j/n, with kappa, omega ~ U(0, 200 pi), phi ~ U(0, 2 pi),
    a_j = j^-alpha (j = 1..n_modes), plus N(0, noise_var), rows centred.

    Built separably (sin(kx - wt + f) = sin(kx) cos(wt - f) - cos(kx) sin(wt - f)),
    column chunk by column chunk, in FP64 before the final rounding.
    Returns the (n, m) contiguous torch tensor At (A = At.T, column-major)."""
    import torch

    dtype = dtype or torch.float32
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    f64 = torch.float64
    J = n_modes
    kappa = torch.rand(J, generator=g, dtype=f64, device=dev) * (200 * math.pi)
    omega = torch.rand(J, generator=g, dtype=f64, device=dev) * (200 * math.pi)
    phi = torch.rand(J, generator=g, dtype=f64, device=dev) * (2 * math.pi)
    amp = torch.arange(1, J + 1, dtype=f64, device=dev) ** (-float(alpha))
    x = torch.arange(m, dtype=f64, device=dev) / m
    t = torch.arange(n, dtype=f64, device=dev) / n
    kx = x[:, None] * kappa[None, :]
    X = torch.cat([torch.sin(kx) * amp, torch.cos(kx) * amp], dim=1)           # m x 2J
    wt = t[:, None] * omega[None, :] - phi[None, :]
    T = torch.cat([torch.cos(wt), -torch.sin(wt)], dim=1)                       # n x 2J
    del kx, wt
    At = torch.empty((n, m), dtype=dtype, device=dev)
    sd = math.sqrt(noise_var)
    rowsum = torch.zeros(m, dtype=f64, device=dev)
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        blk = T[j0:j1] @ X.T
        if sd > 0:
            blk += sd * torch.randn((j1 - j0, m), generator=g, dtype=f64, device=dev)
        At[j0:j1] = blk.to(dtype)
        del blk
    if centre:
        for j0 in range(0, n, chunk):
            rowsum += At[j0:min(n, j0 + chunk)].to(f64).sum(dim=0)
        mu = rowsum / n
        for j0 in range(0, n, chunk):
            j1 = min(n, j0 + chunk)
            At[j0:j1] = (At[j0:j1].to(f64) - mu[None, :]).to(dtype)
    return At


def waves_np(m: int, n: int, n_modes: int, alpha: float, noise_var: float, seed: int,
             centre: bool = True) -> np.ndarray:
    """travelling_waves() on the CPU as an m x n Fortran-ordered FP32 array."""
    At = travelling_waves(m, n, n_modes, alpha, noise_var, seed, centre=centre, device="cpu")
    return np.asfortranarray(At.numpy().T)


@dataclass
class BatchItem:
    m: int
    n: int
    k: int
    c: int
    tau: float
    seed: int


def batch_specs(count: int = 64, seed: int = 1005, m_range=(10_000, 100_000), n_range=(200, 1000),
                k_range=(4, 16), tau_range=(3.0, 12.0)) -> List[BatchItem]:
    """Shapes of the batched workload: m ~ U[10k,100k], n ~ U[200,1000],
    k ~ U[4,16], c = 2k, spectra s_i = exp(-i/tau), tau ~ U[3,12]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        tau = float(rng.uniform(*tau_range))
        out.append(BatchItem(m, n, k, 2 * k, tau, int(rng.integers(0, 2**31 - 1))))
    return out


def batch_matrix(item: BatchItem, dtype=np.float32, noise_var: float = 0.0) -> SpectrumMatrix:
    """One batched-workload matrix: Haar U (m x n), V (n x n), s_i = exp(-i/tau),
    no centring."""
    q = min(item.n, item.m)
    s = np.exp(-np.arange(q) / item.tau)
    return spectrum_matrix(item.m, item.n, s, noise_var, item.seed, centre=False, dtype=dtype,
                           v_orthogonal_to_ones=False)


def batch_matrix_torch(item: BatchItem, device: str = "cuda", dtype=None):
    """batch_matrix() built with torch on `device` (QR of Gaussian matrices in
    FP64, signs fixed so diag(R) > 0), returned as the (n, m) contiguous
    tensor At in `dtype` (default FP32).  For large batches, where the CPU
    QR would take minutes."""
    import torch

    dtype = dtype or torch.float32
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(item.seed))
    f64 = torch.float64

    def haar(rows, cols):
        G = torch.randn((rows, cols), generator=g, dtype=f64, device=dev)
        Q, R = torch.linalg.qr(G)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d[None, :]

    q = min(item.n, item.m)
    s = torch.exp(-torch.arange(q, dtype=f64, device=dev) / item.tau)
    U = haar(item.m, q)
    V = haar(item.n, q)
    At = ((V * s[None, :]) @ U.T).to(dtype).contiguous()
    return At


class WaveBlocks:
    """Column blocks of a travelling-wave matrix (the generator of
    travelling_waves) produced one at a time on `device`: columns [j0, j1) of
    the m x n matrix, t_j = j / n, noise drawn per block from (seed, j0), rows
    centred with means from a pre-pass over all blocks (`centre`)."""

    def __init__(self, m: int, n: int, n_modes: int, alpha: float, noise_var: float, seed: int,
                 device: str = "cuda", centre: bool = True, chunk: int = 512):
        import torch

        self.m, self.n, self.seed, self.dev = m, n, seed, torch.device(device)
        self.sd = math.sqrt(noise_var)
        f64 = torch.float64
        g = torch.Generator(device=self.dev)
        g.manual_seed(int(seed))
        J = n_modes
        kappa = torch.rand(J, generator=g, dtype=f64, device=self.dev) * (200 * math.pi)
        self.omega = torch.rand(J, generator=g, dtype=f64, device=self.dev) * (200 * math.pi)
        self.phi = torch.rand(J, generator=g, dtype=f64, device=self.dev) * (2 * math.pi)
        amp = torch.arange(1, J + 1, dtype=f64, device=self.dev) ** (-float(alpha))
        x = torch.arange(m, dtype=f64, device=self.dev) / m
        kx = x[:, None] * kappa[None, :]
        self.X = torch.cat([torch.sin(kx) * amp, torch.cos(kx) * amp], dim=1)
        self.mu = None
        if centre:
            rowsum = torch.zeros(m, dtype=f64, device=self.dev)
            for j0 in range(0, n, chunk):
                rowsum += self._raw(j0, min(n, j0 + chunk)).sum(dim=0)
            self.mu = rowsum / n

    def _raw(self, j0: int, j1: int):
        import torch

        t = torch.arange(j0, j1, dtype=torch.float64, device=self.dev) / self.n
        wt = t[:, None] * self.omega[None, :] - self.phi[None, :]
        T = torch.cat([torch.cos(wt), -torch.sin(wt)], dim=1)
        blk = T @ self.X.T
        if self.sd > 0:
            g = torch.Generator(device=self.dev)
            g.manual_seed(int(self.seed) * 1_000_003 + j0)
            blk += self.sd * torch.randn(blk.shape, generator=g, dtype=torch.float64, device=self.dev)
        return blk

    def block(self, j0: int, j1: int, dtype=None):
        """(j1 - j0, m) contiguous tensor: row j is column j0 + j of A."""
        import torch

        blk = self._raw(j0, j1)
        if self.mu is not None:
            blk -= self.mu[None, :]
        return blk.to(dtype or torch.float32)
