"""Preprocessing on the GPU through the C ABI, against the oracle:
  * per-gene moments (int64 sums of x and x^2) bit-exact on the 68k-cell
    recipe, and the standard deviations from them within 1e-12 of numpy;
  * the CSR restricted to the 200 genes of largest standard deviation,
    bit-exact (row offsets, renumbered genes, counts);
  * end to end: a 10x Market Matrix file of the small recipe, read, reduced
    to its 300 most variable genes and clustered from one cluster, recovers
    the four clusters."""
import gzip
import io
import os
import sys

import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp

import oracle
from paper_1812_10048_amd import prep, quality, synth
from paper_1812_10048_amd.sampler import Sampler

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def exact_top(s, q, n, k):
    """The k genes of largest variance (n sum x^2 - (sum x)^2) / n^2, in exact
    integers; equal variances: the lower gene first; in increasing order."""
    b = [int(n) * int(qi) - int(si) * int(si) for si, qi in zip(s, q)]
    order = sorted(range(len(b)), key=lambda u: (-b[u], u))
    return np.sort(np.array(order[: min(k, len(b))], dtype=np.int64))


def test_top_genes_ties_go_to_the_lower_gene():
    """Genes 1 and 3 have the same counts in every cell, as have 2 and 5: equal
    variances, which the exact ranking orders by gene index."""
    rng = np.random.default_rng(4)
    X = rng.integers(0, 5, size=(300, 7))
    X[:, 3] = X[:, 1] * 3
    X[:, 1] = X[:, 3]
    X[:, 5] = X[:, 2]
    X[:, 0] = 0
    d = synth.from_dense(X)
    rp, col, val = d.host_arrays()
    rs, rq = oracle.gene_moments(rp, col, val, d.n_genes)
    for k in range(0, 9):
        genes, gmap, _ = prep.top_genes(rp, col, val, d.n_genes, k)
        assert np.array_equal(genes, exact_top(rs, rq, d.n_cells, k)), k


def test_gene_moments_and_filter_match_the_oracle():
    _say("prep c2")
    d = synth.generate("c2", seed=0)
    rp, col, val = d.host_arrays()
    s, q = prep.gene_moments(rp, col, val, d.n_genes)
    rs, rq = oracle.gene_moments(rp, col, val, d.n_genes)
    assert np.array_equal(s.astype(np.int64), rs) and np.array_equal(q.astype(np.int64), rq)
    genes, gmap, std = prep.top_genes(rp, col, val, d.n_genes, 200)
    n = d.n_cells
    ref_std = np.sqrt((n * rq.astype(np.float64) - rs.astype(np.float64) ** 2) / n ** 2)
    assert np.allclose(std, ref_std, rtol=1e-12, atol=1e-12)
    assert np.array_equal(genes, exact_top(rs, rq, n, 200))
    m = gmap.cpu().numpy()
    assert np.array_equal(m[genes], np.arange(genes.size)) and np.all(np.delete(m, genes) == -1)
    grp, gcol, gval = prep.filter_genes(rp, col, val, d.n_genes, gmap)
    orp, ocol, oval = oracle.filter_csr(rp, col, val, genes)
    assert np.array_equal(grp.cpu().numpy(), orp)
    assert np.array_equal(gcol.cpu().numpy(), ocol) and np.array_equal(gval.cpu().numpy(), oval)


def test_10x_file_to_clusters(tmp_path):
    _say("prep 10x end to end")
    d = synth.generate("c1", seed=0)
    rp, col, val = d.host_arrays()
    m = sp.csr_matrix((val, col, rp), shape=(d.n_cells, d.n_genes)).T.tocoo()   # features x barcodes
    buf = io.BytesIO()
    scipy.io.mmwrite(buf, m, field="integer")
    path = os.path.join(tmp_path, "matrix.mtx.gz")
    with gzip.open(path, "wb") as f:
        f.write(buf.getvalue())
    rp2, col2, val2, G, N = prep.read_10x_mtx(path)
    assert (G, N) == (d.n_genes, d.n_cells)
    genes, gmap, _ = prep.top_genes(rp2, col2, val2, G, 300)
    frp, fcol, fval = prep.filter_genes(rp2, col2, val2, G, gmap)
    s = Sampler(frp, fcol, fval, len(genes), seed=0, k_max=32, precision="fp32")
    for _ in range(30):
        s.sweep(1)
        s.split_merge()
    c, _ = s.labels()
    ari = quality.adjusted_rand_index(d.z, c.cpu().numpy())
    _say("ARI", ari, "K", s.stats()["K"])
    assert ari > 0.95 and s.stats()["K"] == 4
