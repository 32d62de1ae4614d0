"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds random-number generation only -- none of the emulation's
arithmetic -- so that the CPU oracle and the GPU library can be fed the very
same bits without sharing any code.

Generator of the paper's evaluation (Sec. V-B, Eq. 19):
    a_ij = (u - 0.5) * exp(phi * g),   u ~ U(0, 1),  g ~ N(0, 1),
where phi widens the exponent range (the paper uses phi = 4).  Draws use
numpy's PCG64 in float64 on the host.

Seed rule: seed = 1_000_003*cfg + 10_007*n + 101*round(10*phi) + role + rep,
role 0 = A, 1 = B, 2 = imaginary part of A, 3 = imaginary part of B.
"""
from __future__ import annotations

import numpy as np

ROLE_A, ROLE_B, ROLE_A_IM, ROLE_B_IM = 0, 1, 2, 3


def seed_for(cfg: int, n: int, phi: float, role: int, rep: int = 0) -> int:
    return 1_000_003 * cfg + 10_007 * n + 101 * int(round(10 * phi)) + role + rep


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def phi_matrix(rows: int, cols: int, phi: float, seed: int) -> np.ndarray:
    """(u - 0.5) * exp(phi * g), float64, C order."""
    r = _rng(seed)
    u = r.random((rows, cols))
    g = r.standard_normal((rows, cols))
    return (u - 0.5) * np.exp(phi * g)


def uniform_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """Entries uniform in (-1, 1): 2u - 1."""
    return 2.0 * _rng(seed).random((rows, cols)) - 1.0


def complex_phi_matrix(rows: int, cols: int, phi: float, seed_re: int, seed_im: int) -> np.ndarray:
    """Real and imaginary parts drawn independently from the phi generator."""
    return phi_matrix(rows, cols, phi, seed_re) + 1j * phi_matrix(rows, cols, phi, seed_im)


def short_mantissa_matrix(rows: int, cols: int, bits: int, seed: int,
                          emin: int = -8, emax: int = 8) -> np.ndarray:
    """Entries m * 2^e with |m| < 2^bits an integer and e uniform in [emin, emax]:
    few enough significant bits that the product can be exact."""
    r = _rng(seed)
    m = r.integers(-(2 ** bits) + 1, 2 ** bits, size=(rows, cols))
    e = r.integers(emin, emax + 1, size=(rows, cols))
    return np.ldexp(m.astype(np.float64), e)


def log_uniform_ints(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Integers distributed log-uniformly in [lo, hi] (batch problem sizes)."""
    r = _rng(seed)
    x = np.exp(r.uniform(np.log(lo), np.log(hi + 1), size=count))
    return np.clip(np.floor(x).astype(np.int64), lo, hi)


def with_structure(X: np.ndarray, seed: int, zero_rows=(), zero_cols=(),
                   scale_rows=None) -> np.ndarray:
    """Copy of X with chosen rows/columns zeroed and rows rescaled by powers of
    two (scale_rows: dict row -> exponent), for edge-case parity inputs."""
    Y = np.array(X, copy=True)
    for i in zero_rows:
        Y[i, :] = 0
    for j in zero_cols:
        Y[:, j] = 0
    if scale_rows:
        for i, e in scale_rows.items():
            Y[i, :] = np.ldexp(Y[i, :], e)
    return Y


def phi_matrix_device(rows: int, cols: int, phi: float, seed: int, device="cuda:0"):
    """The same distribution drawn on the GPU with torch's seeded generator
    (for full-size problems; tests copy the rows and columns they check back
    to the host, so both sides see identical bits).  Returns a float64
    torch tensor."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    u = torch.rand((rows, cols), generator=g, dtype=torch.float64, device=device)
    n = torch.randn((rows, cols), generator=g, dtype=torch.float64, device=device)
    return (u - 0.5) * torch.exp(phi * n)
