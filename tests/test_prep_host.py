"""Preprocessing on the host (no GPU): 10x Market Matrix reading against
scipy's writer, the top-k gene choice with its tie rule, and the oracle's
moments and restricted CSR against numpy and scipy.sparse."""
import gzip
import io
import os

import numpy as np
import pytest
import scipy.io
import scipy.sparse as sp

import oracle
from paper_1812_10048_amd import prep


def _random_counts(rng, n_genes, n_cells, density=0.2):
    m = sp.random(n_genes, n_cells, density=density, random_state=np.random.RandomState(int(rng.integers(1 << 30))),
                  data_rvs=lambda k: rng.integers(1, 300, size=k)).tocoo()
    return sp.coo_matrix((m.data.astype(np.int64), (m.row, m.col)), shape=m.shape)


@pytest.mark.parametrize("gz", [False, True])
def test_read_10x_mtx_matches_scipy(tmp_path, gz):
    rng = np.random.default_rng(0)
    m = _random_counts(rng, 37, 53)
    buf = io.BytesIO()
    scipy.io.mmwrite(buf, m, field="integer")
    path = os.path.join(tmp_path, "matrix.mtx" + (".gz" if gz else ""))
    with (gzip.open(path, "wb") if gz else open(path, "wb")) as f:
        f.write(buf.getvalue())
    rp, col, val, G, N = prep.read_10x_mtx(path)
    ref = m.T.tocsr()
    ref.sort_indices()
    assert (G, N) == (37, 53)
    assert np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices) and np.array_equal(val, ref.data)


def test_read_10x_mtx_rejects_bad_files(tmp_path):
    p = os.path.join(tmp_path, "bad.mtx")
    with open(p, "w") as f:
        f.write("%%MatrixMarket matrix coordinate real general\n2 2 1\n1 1 1.5\n")
    with pytest.raises(ValueError):
        prep.read_10x_mtx(p)
    with open(p, "w") as f:
        f.write("%%MatrixMarket matrix coordinate integer general\n2 2 2\n1 1 3\n1 1 4\n")
    with pytest.raises(ValueError):
        prep.read_10x_mtx(p)


def test_oracle_moments_and_filter_against_numpy_and_scipy():
    rng = np.random.default_rng(1)
    m = _random_counts(rng, 40, 70).T.tocsr()
    m.sort_indices()
    dense = m.toarray()
    s, q = oracle.gene_moments(m.indptr, m.indices, m.data, 40)
    assert np.array_equal(s, dense.sum(axis=0)) and np.array_equal(q, (dense ** 2).sum(axis=0))
    n = dense.shape[0]
    std = np.sqrt((n * q - s * s) / n ** 2)
    assert np.allclose(std, dense.std(axis=0), rtol=1e-12, atol=0)
    genes = np.array([0, 3, 7, 8, 20, 39])
    rp, col, val = oracle.filter_csr(m.indptr, m.indices, m.data, genes)
    ref = m[:, genes].tocsr()
    ref.sort_indices()
    ref.eliminate_zeros()
    assert np.array_equal(rp, ref.indptr) and np.array_equal(col, ref.indices) and np.array_equal(val, ref.data)
