"""Seeded synthetic tensors shaped like the paper's workloads.

This module only makes inputs.  It is shared by the tests, the benchmark and
the smoke check, and it holds none of the compression method's arithmetic:
the planted tensor is assembled with ``torch.tensordot`` (a library
contraction) and every random number comes from a seeded ``torch.Generator``.

Recipe (used for every workload):

* core ``G = Z * (d_1 o ... o d_N)`` with ``Z`` iid N(0,1) and
  ``d_n(r) = rho**r`` for ``r = 0..R_n-1`` (``rho = 1``: no decay);
* factors with orthonormal columns, either the Q factor of a seeded Gaussian
  ``I_n x R_n`` matrix (``"gaussian"``), or a smooth cosine basis
  ``cos(pi (i + 1/2) r / I_n)`` plus a seeded perturbation
  ``delta * N(0,1) / sqrt(I_n)`` (``"cosine"``), orthonormalised by QR with a
  positive diagonal in R;
* ``X0 = G x_1 U_1 ... x_N U_N`` in FP64, so ``||X0|| = ||G||``;
* Gaussian noise, either rescaled to exactly ``eta * ||X0||`` (``"exact"``) or
  with standard deviation ``eta * ||G|| / sqrt(#X)`` (``"sigma"``).

Tensors are returned with logical shape ``(I_1, ..., I_N)`` and mode 1
fastest in memory (Fortran strides), the layout of the paper's local
tensors.  Tensors above 32 GB in FP64 are built one slab of the last mode at
a time (same recipe, the noise drawn slab after slab).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Sequence

import torch

__all__ = [
    "Workload",
    "WORKLOADS",
    "batch_workload",
    "planted_tucker",
    "fortran_empty",
    "is_fortran",
    "random_tensor",
]


def fortran_empty(dims: Sequence[int], dtype=torch.float64, device="cpu") -> torch.Tensor:
    """Uninitialised tensor of logical shape ``dims`` with mode 1 fastest."""
    n = len(dims)
    t = torch.empty(tuple(reversed(list(dims))), dtype=dtype, device=device)
    return t.permute(*reversed(range(n)))


def is_fortran(x: torch.Tensor) -> bool:
    """True when ``x`` is densely packed with dimension 0 fastest."""
    expect = 1
    for d, s in zip(x.shape, x.stride()):
        if d != 1 and s != expect:
            return False
        expect *= d
    return True


def _to_fortran(c_order: torch.Tensor) -> torch.Tensor:
    """View a C-contiguous tensor of shape (I_N..I_1) as logical (I_1..I_N)."""
    return c_order.permute(*reversed(range(c_order.dim())))


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _orthonormal(a: torch.Tensor) -> torch.Tensor:
    q, r = torch.linalg.qr(a)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1
    return q * d.unsqueeze(0)


def _factor(i_n: int, r_n: int, kind: str, delta: float, g, device) -> torch.Tensor:
    if kind == "gaussian":
        a = torch.randn(i_n, r_n, generator=g, dtype=torch.float64, device=device)
    elif kind == "cosine":
        i = torch.arange(i_n, dtype=torch.float64, device=device).unsqueeze(1)
        r = torch.arange(r_n, dtype=torch.float64, device=device).unsqueeze(0)
        a = torch.cos(math.pi * (i + 0.5) * r / i_n)
        a = a + delta * torch.randn(i_n, r_n, generator=g, dtype=torch.float64,
                                    device=device) / math.sqrt(i_n)
    else:
        raise ValueError(f"unknown factor kind {kind!r}")
    return _orthonormal(a)


def planted_tucker(dims: Sequence[int], ranks: Sequence[int], *, rho: float = 1.0,
                   factor_kind: str = "gaussian", delta: float = 0.1, noise: float = 0.0,
                   noise_mode: str = "exact", seed: int = 0, dtype=torch.float64,
                   device="cpu", return_parts: bool = False):
    """Planted multilinear-rank tensor plus Gaussian noise (see module doc).

    Returns a Fortran-strided tensor of logical shape ``dims`` in ``dtype``
    (built in FP64, rounded to nearest even once at the end).  With
    ``return_parts`` also returns ``(core, factors)`` in FP64.
    """
    dims = [int(d) for d in dims]
    ranks = [int(r) for r in ranks]
    if len(dims) != len(ranks) or any(r < 1 or r > d for r, d in zip(ranks, dims)):
        raise ValueError("ranks must satisfy 1 <= R_n <= I_n")
    n = len(dims)
    dev = torch.device(device)
    g = _gen(seed, dev)
    factors = [_factor(dims[k], ranks[k], factor_kind, delta, g, dev) for k in range(n)]
    core_c = torch.randn(tuple(reversed(ranks)), generator=g, dtype=torch.float64, device=dev)
    for k in range(n):
        scale = rho ** torch.arange(ranks[k], dtype=torch.float64, device=dev)
        shape = [1] * n
        shape[n - 1 - k] = ranks[k]
        core_c = core_c * scale.view(shape)
    if math.prod(dims) * 8 > _SLAB_BYTES and not return_parts:
        return _planted_by_slabs(dims, ranks, factors, core_c, noise, noise_mode, g, dtype, dev)
    # X0 = G x_1 U_1 ... x_N U_N; mode k is axis n-1-k of the C-order array.
    t = core_c
    for k in sorted(range(n), key=lambda m: dims[m] / ranks[m]):
        ax = n - 1 - k
        t = torch.tensordot(t, factors[k], dims=([ax], [1]))  # new axis appended last
        t = torch.movedim(t, -1, ax).contiguous()
    x_c = t
    core_norm = torch.linalg.vector_norm(core_c).item()
    if noise > 0:
        total = x_c.numel()
        if noise_mode == "exact":
            e = torch.randn(x_c.shape, generator=g, dtype=torch.float64, device=dev)
            x0_norm = torch.linalg.vector_norm(x_c).item()
            e_norm = torch.linalg.vector_norm(e).item()
            x_c.add_(e, alpha=noise * x0_norm / e_norm)
            del e
        elif noise_mode == "sigma":
            sigma = noise * core_norm / math.sqrt(total)
            # chunk over the slowest mode to bound the temporary
            flat = x_c.view(x_c.shape[0], -1)
            step = max(1, (1 << 27) // max(1, flat.shape[1]))
            for s in range(0, flat.shape[0], step):
                blk = flat[s:s + step]
                blk.add_(torch.randn(blk.shape, generator=g, dtype=torch.float64, device=dev),
                         alpha=sigma)
        else:
            raise ValueError(f"unknown noise mode {noise_mode!r}")
    out = _to_fortran(x_c if dtype == torch.float64 else x_c.to(dtype))
    if return_parts:
        core = _to_fortran(core_c)
        return out, core, factors
    return out


# Tensors whose FP64 form exceeds this are built one last-mode slab at a time.
_SLAB_BYTES = 1 << 35


def _planted_by_slabs(dims, ranks, factors, core_c, noise, noise_mode, g, dtype, dev):
    """``planted_tucker`` for tensors too large to hold in FP64 (with its
    temporaries): slab t of the last mode is ``(G x_N U_N[t, :]) x_1 U_1 ...
    x_{N-1} U_{N-1}``, formed in FP64, given its noise, rounded once to
    ``dtype`` and stored; the noise comes from the same generator, slab after
    slab.  Only ``noise_mode="sigma"`` applies (``"exact"`` needs the whole
    tensor's norm first)."""
    if noise > 0 and noise_mode != "sigma":
        raise ValueError("slab-wise generation supports noise_mode='sigma' only")
    n = len(dims)
    out = fortran_empty(dims, dtype, dev)
    out_c = out.permute(*reversed(range(n)))          # C order (I_N, ..., I_1), contiguous
    sigma = noise * torch.linalg.vector_norm(core_c).item() / math.sqrt(math.prod(dims))
    order = sorted(range(n - 1), key=lambda m: dims[m] / ranks[m])
    for t in range(dims[n - 1]):
        s = torch.tensordot(factors[n - 1][t], core_c, dims=([0], [0]))  # (R_{N-1}, ..., R_1)
        for k in order:
            ax = n - 2 - k
            s = torch.tensordot(s, factors[k], dims=([ax], [1]))
            s = torch.movedim(s, -1, ax).contiguous()
        if noise > 0:
            s.add_(torch.randn(s.shape, generator=g, dtype=torch.float64, device=dev),
                   alpha=sigma)
        out_c[t].copy_(s)
        del s
    return out


def random_tensor(dims: Sequence[int], *, seed: int = 0, dtype=torch.float64,
                  device="cpu") -> torch.Tensor:
    """Plain iid N(0,1) tensor (no structure), Fortran strides."""
    g = _gen(seed, torch.device(device))
    c = torch.randn(tuple(reversed([int(d) for d in dims])), generator=g,
                    dtype=torch.float64, device=device)
    return _to_fortran(c if dtype == torch.float64 else c.to(dtype))


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: shape, planted ranks and generator settings."""
    name: str
    dims: tuple
    ranks: tuple
    rho: float
    factor_kind: str
    noise: float
    noise_mode: str
    eps: float
    seed: int
    order: tuple = field(default=None)

    def make(self, dtype=torch.float64, device="cpu", seed=None, return_parts=False):
        return planted_tucker(self.dims, self.ranks, rho=self.rho,
                              factor_kind=self.factor_kind, noise=self.noise,
                              noise_mode=self.noise_mode,
                              seed=self.seed if seed is None else seed, dtype=dtype,
                              device=device, return_parts=return_parts)

    @property
    def numel(self) -> int:
        return math.prod(self.dims)


WORKLOADS = {
    # small 3-way case the CPU oracle finishes in seconds
    "planted32": Workload("planted32", (32, 32, 32), (4, 5, 6), 1.0, "gaussian", 1e-6,
                          "exact", 1e-4, 1),
    # combustion-shaped 5-way: 3 spatial x 32 variables x 32 time steps
    "combustion128": Workload("combustion128", (128, 128, 128, 32, 32), (16, 16, 16, 8, 8),
                              0.7, "cosine", 1e-5, "sigma", 1e-4, 2),
    # one GPU's share of an SP-sized dataset
    "combustion256": Workload("combustion256", (256, 256, 256, 64, 16), (32, 32, 32, 16, 8),
                              0.8, "cosine", 1e-5, "sigma", 1e-4, 5),
}


def batch_workload(count: int = 64, seed: int = 4000, smin: int = 24, smax: int = 96,
                   nvar: int = 16, ranks=(12, 12, 12, 6), rho: float = 0.6,
                   noise: float = 1e-5, eps: float = 1e-4):
    """A batch of uneven combustion-shaped problems: problem t is s^3 x nvar
    with s drawn uniformly from [smin, smax] (seeded), planted ranks capped by
    the extents, cosine factors, geometric decay rho, noise as a per-element
    sigma, generator seed seed + t.  Returns a list of Workload."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = rng.integers(smin, smax + 1, size=count)
    out = []
    for t, s in enumerate(sizes):
        s = int(s)
        dims = (s, s, s, nvar)
        rk = tuple(min(r, d) for r, d in zip(ranks, dims))
        out.append(Workload(f"batch{t}", dims, rk, rho, "cosine", noise, "sigma", eps,
                            seed + t))
    return out
