"""Clustering quality of the sampler against the synthetic truth.

Section 4 scores clusterings by the adjusted Rand index, the Rand index and
the Hubert index against known labels.  Its data sets are not available; the
seeded recipes of ``synth`` stand in for them, with their true clusters as
the reference.  The sampler starts from one cluster and runs
(sweep, split/merge) iterations on the GPU; the labels are scored every few
iterations.

    python -m paper_1812_10048_amd.quality --config c2 --iters 200 --alpha 0.1 0.5 1

prints one JSON line per scored iteration.  ``--lib-mean`` reruns the recipe at
other mean library sizes (Section 4 relates clustering quality to sequencing
depth), and ``--conc`` changes the Dirichlet concentration of the true
profiles (larger is closer clusters, a harder problem).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def _pairs(x: np.ndarray) -> float:
    x = x.astype(np.float64)
    return float(np.sum(x * (x - 1.0) / 2.0))


def pair_counts(a, b) -> tuple[float, float, float, float]:
    """(pairs together in both, sum of C(row sums, 2), sum of C(column sums, 2),
    C(n, 2)) of the contingency table of two labelings."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    if a.shape != b.shape:
        raise ValueError("labelings of different lengths")
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    nb = int(bi.max()) + 1 if bi.size else 1
    table = np.bincount(ai * nb + bi).astype(np.float64)
    n = float(a.size)
    return _pairs(table), _pairs(np.bincount(ai)), _pairs(np.bincount(bi)), n * (n - 1.0) / 2.0


def rand_index(a, b) -> float:
    """Fraction of cell pairs on which the two labelings agree (together in
    both or apart in both)."""
    nij, na, nb, m = pair_counts(a, b)
    if m == 0:
        return 1.0
    return (m + 2.0 * nij - na - nb) / m


def adjusted_rand_index(a, b) -> float:
    """Rand index corrected for chance (Hubert and Arabie): 1 for identical
    partitions, 0 in expectation for independent ones."""
    nij, na, nb, m = pair_counts(a, b)
    if m == 0:
        return 1.0
    expected = na * nb / m
    top = 0.5 * (na + nb) - expected
    if top == 0.0:
        return 1.0
    return (nij - expected) / top


def hubert_index(a, b) -> float:
    """Agreeing minus disagreeing pairs over all pairs, 2 RI - 1."""
    return 2.0 * rand_index(a, b) - 1.0


def recipe_variant(config: str, lib_mean: float | None = None, conc: float | None = None):
    """The named recipe with its mean library size and/or profile
    concentration replaced, named after the change."""
    import dataclasses

    from . import synth

    r = synth.RECIPES[config]
    name = r.name
    if lib_mean is not None:
        r = dataclasses.replace(r, lib_mean=float(lib_mean))
        name += f"-lib{lib_mean:g}"
    if conc is not None:
        r = dataclasses.replace(r, conc=float(conc))
        name += f"-conc{conc:g}"
    return dataclasses.replace(r, name=name)


def run(config: str, iters: int, alpha: float, precision: str, seed: int, every: int, k_max: int,
        split_q: bool, new_cluster: bool, data=None, extra=None):
    import torch

    from . import synth
    from .sampler import Sampler

    d = data if data is not None else synth.generate(config, seed=seed, device="cuda")
    s = Sampler(d.row_ptr, d.col, d.val, d.n_genes, alpha=alpha, beta=1.0, seed=seed, k_init=1,
                k_max=k_max, precision=precision, split_q=split_q, new_cluster=new_cluster)
    out = []
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        s.sweep(1)
        s.split_merge()
        if it % every == 0 or it == iters:
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            c, _ = s.labels()
            c = c.cpu().numpy()
            rec = dict(config=config, **(extra or {}), alpha=alpha, precision=precision, iter=it, K=int(s.stats()["K"]),
                       ari=adjusted_rand_index(d.z, c), ri=rand_index(d.z, c), hi=hubert_index(d.z, c),
                       seconds=round(el, 3))
            out.append(rec)
            print(json.dumps(rec), flush=True)
            t0 = time.perf_counter() - el   # exclude the scoring from the clock
    s.close()
    return out


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--alpha", type=float, nargs="+", default=[1.0])
    ap.add_argument("--precision", default="split_bf16")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--k-max", type=int, default=128)
    ap.add_argument("--split-q", action="store_true")
    ap.add_argument("--new-cluster", action="store_true")
    ap.add_argument("--lib-mean", type=float, nargs="+", default=None)
    ap.add_argument("--conc", type=float, default=None)
    a = ap.parse_args()
    from . import synth
    for lib in (a.lib_mean or [None]):
        rec = recipe_variant(a.config, lib, a.conc)
        data = synth.generate(rec, seed=a.seed, device="cuda")
        extra = dict(lib_mean=rec.lib_mean, conc=rec.conc, zeros=round(data.zero_fraction(), 4))
        for alpha in a.alpha:
            run(rec.name, a.iters, alpha, a.precision, a.seed, a.every, a.k_max, a.split_q, a.new_cluster, data,
                extra)


if __name__ == "__main__":
    main()
