"""Seeded synthetic UMI count matrices shaped like droplet scRNA-seq data.

This module only generates inputs: it holds none of the sampler's arithmetic
and is shared, as a data source, by the GPU library's tests and benchmark and
by the CPU oracle's tests.

Recipe (the paper's 10x data, Sections 3 and 4, is not available; these
matrices stand in for it): ``K`` true clusters with given sizes, cluster
profiles theta_k ~ Dirichlet(conc * 1_G), library sizes
L_i = max(1, round(LogNormal(mu, sigma))) with mu = ln(mean) - sigma^2 / 2 so
that E[L] = mean, and counts x_i ~ Multinomial(L_i, theta_{z_i}) (eq. 26).
Cells are generated cluster by cluster and then shuffled with the seed.

The small parameters (sizes, profiles, library sizes, the shuffle) come from
``numpy.random.default_rng(seed)``; the multinomial draws, the only heavy
part, come from a ``torch.Generator`` on the requested device, by inverse-CDF
sampling of L_i categorical draws per cell.  A given (config, seed, device
type) always yields the same matrix.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch


@dataclasses.dataclass
class Recipe:
    name: str
    n_cells: int
    n_genes: int
    sizes: str            # "fixed:<a,b,...>" | "dirichlet:<K>" | "powerlaw:<K>:<exponent>"
    conc: float           # Dirichlet concentration of the true profiles
    lib_mean: float       # mean library size (UMIs per cell)
    lib_sigma: float      # log-scale sigma of the library size


RECIPES = {
    # 2k cells x 500 genes, 4 clusters of 800/600/400/200 cells
    "c1": Recipe("c1", 2_000, 500, "fixed:800,600,400,200", 0.1, 1500.0, 0.5),
    # 68k cells x 1,000 genes, 10 clusters with Dirichlet(1) sizes
    "c2": Recipe("c2", 68_000, 1_000, "dirichlet:10", 0.05, 2000.0, 0.6),
    # 100k cells x 2,000 genes, 12 power-law clusters (the 1.3M recipe, smaller)
    "c4": Recipe("c4", 100_000, 2_000, "powerlaw:12:1.5", 0.03, 3000.0, 0.7),
    # 1.3M cells x 2,000 genes, 40 power-law clusters
    "c5": Recipe("c5", 1_300_000, 2_000, "powerlaw:40:1.5", 0.03, 3000.0, 0.7),
}


@dataclasses.dataclass
class Dataset:
    name: str
    n_cells: int
    n_genes: int
    row_ptr: torch.Tensor   # int64 [N+1]
    col: torch.Tensor       # int32 [nnz], sorted within each row
    val: torch.Tensor       # int32 [nnz], >= 1
    z: np.ndarray           # int64 [N] true cluster of each cell
    n_true: int

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def zero_fraction(self) -> float:
        return 1.0 - self.nnz / (self.n_cells * self.n_genes)

    def to(self, device) -> "Dataset":
        return dataclasses.replace(self, row_ptr=self.row_ptr.to(device), col=self.col.to(device),
                                   val=self.val.to(device))

    def host_arrays(self, cells: int | None = None):
        """(row_ptr, col, val) as numpy, optionally only the first ``cells`` rows."""
        rp = self.row_ptr.cpu().numpy()
        if cells is None or cells >= self.n_cells:
            return rp, self.col.cpu().numpy(), self.val.cpu().numpy()
        end = int(rp[cells])
        return rp[: cells + 1].copy(), self.col[:end].cpu().numpy(), self.val[:end].cpu().numpy()


def _largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    w = np.asarray(weights, dtype=np.float64)
    exact = w / w.sum() * total
    base = np.floor(exact).astype(np.int64)
    rem = total - int(base.sum())
    order = np.argsort(-(exact - base), kind="stable")
    base[order[:rem]] += 1
    return base


def cluster_sizes(spec: str, n_cells: int, rng: np.random.Generator) -> np.ndarray:
    kind, _, rest = spec.partition(":")
    if kind == "fixed":
        sizes = np.array([int(v) for v in rest.split(",")], dtype=np.int64)
        assert int(sizes.sum()) == n_cells
        return sizes
    if kind == "dirichlet":
        K = int(rest)
        return _largest_remainder(rng.dirichlet(np.ones(K)), n_cells)
    if kind == "powerlaw":
        K, expo = rest.split(":")
        K = int(K)
        w = np.arange(1, K + 1, dtype=np.float64) ** (-float(expo))
        return _largest_remainder(w, n_cells)
    raise ValueError(spec)


def generate(recipe: Recipe | str, seed: int = 0, device="cpu", n_cells: int | None = None,
             chunk_draws: int = 200_000_000) -> Dataset:
    """Generate the recipe's count matrix; ``n_cells`` overrides the cell count
    (sizes are rescaled by largest remainder)."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    N = int(n_cells or recipe.n_cells)
    G = recipe.n_genes
    rng = np.random.default_rng(seed)
    if n_cells is None:
        sizes = cluster_sizes(recipe.sizes, N, rng)
    else:
        sizes = _largest_remainder(cluster_sizes(recipe.sizes, recipe.n_cells, rng).astype(np.float64), N)
    K = sizes.size
    theta = rng.dirichlet(np.full(G, recipe.conc), size=K)             # [K, G]
    z = np.repeat(np.arange(K, dtype=np.int64), sizes)
    z = z[rng.permutation(N)]
    mu = math.log(recipe.lib_mean) - 0.5 * recipe.lib_sigma ** 2
    lib = np.maximum(1, np.rint(rng.lognormal(mu, recipe.lib_sigma, size=N))).astype(np.int64)

    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1_000_003 + 17)
    # cumulative profiles, cluster k shifted into [k, k+1) so one sorted array serves all
    cdf = np.cumsum(theta, axis=1)
    cdf /= cdf[:, -1:]
    cdf[:, -1] = 1.0
    shifted = torch.from_numpy((cdf + np.arange(K)[:, None]).reshape(-1)).to(dev)
    z_t = torch.from_numpy(z).to(dev)
    lib_t = torch.from_numpy(lib).to(dev)

    row_counts = []
    cols = []
    vals = []
    start = 0
    csum = np.cumsum(lib)
    while start < N:
        # as many cells as fit in the draw budget (at least one)
        base = csum[start - 1] if start > 0 else 0
        end = int(np.searchsorted(csum, base + chunk_draws, side="right"))
        end = max(end, start + 1)
        end = min(end, N)
        n = end - start
        L = lib_t[start:end]
        cell = torch.repeat_interleave(torch.arange(n, device=dev), L)
        u = torch.rand(cell.numel(), generator=gen, device=dev, dtype=torch.float64)
        u = u + z_t[start:end][cell].to(torch.float64)
        idx = torch.searchsorted(shifted, u, right=True)
        gene = idx - z_t[start:end][cell] * G
        gene = gene.clamp_(0, G - 1)
        dense = torch.bincount(cell * G + gene, minlength=n * G).view(n, G)
        nz = dense.nonzero(as_tuple=False)
        row_counts.append(torch.bincount(nz[:, 0], minlength=n))
        cols.append(nz[:, 1].to(torch.int32))
        vals.append(dense[nz[:, 0], nz[:, 1]].to(torch.int32))
        del dense, cell, u, idx, gene, nz
        start = end
    counts = torch.cat(row_counts)
    row_ptr = torch.zeros(N + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return Dataset(recipe.name, N, G, row_ptr, torch.cat(cols), torch.cat(vals), z, K)


def from_dense(x: np.ndarray, name: str = "dense") -> Dataset:
    """Wrap a small dense [N, G] integer matrix as a Dataset (for tests)."""
    x = np.asarray(x, dtype=np.int64)
    N, G = x.shape
    rows, cols = np.nonzero(x)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Dataset(name, N, G, torch.from_numpy(row_ptr), torch.from_numpy(cols.astype(np.int32)),
                   torch.from_numpy(x[rows, cols].astype(np.int32)), np.zeros(N, dtype=np.int64), 1)
