"""Preprocessing before the sampler.

Section 3 clusters droplet UMI data after keeping the genes of largest
standard deviation across cells.  This module reads 10x Market Matrix files
into the cell-major CSR the library takes, ranks the genes by standard
deviation exactly on the GPU from the per-gene moments (the library's HIP
kernels), and restricts the CSR to the chosen genes on the GPU.  Reading files is host
IO; every pass over the counts runs in the library.
"""
from __future__ import annotations

import gzip

import numpy as np
import torch

from . import dpmm as C


def read_10x_mtx(path: str):
    """A Matrix Market ``coordinate integer`` file as written by 10x (rows are
    features, columns are barcodes, 1-based; ``.gz`` is read through gzip)
    into a cell-major CSR: (row_ptr int64[N+1], col int32, val int32, n_genes,
    n_cells), columns sorted within each row, zero counts dropped."""
    opener = gzip.open if path.endswith(".gz") else open
    with opener(path, "rt") as f:
        header = f.readline().split()
        if len(header) < 4 or header[0] != "%%MatrixMarket" or header[1] != "matrix" or header[2] != "coordinate":
            raise ValueError(f"{path}: not a Matrix Market coordinate file")
        if header[3] != "integer":
            raise ValueError(f"{path}: counts must be integer, not {header[3]}")
        if len(header) > 4 and header[4] != "general":
            raise ValueError(f"{path}: only the general symmetry is supported")
        line = f.readline()
        while line.startswith("%"):
            line = f.readline()
        n_genes, n_cells, nnz = (int(v) for v in line.split())
        data = np.array(f.read().split(), dtype=np.int64)
    if data.size != 3 * nnz:
        raise ValueError(f"{path}: {data.size // 3} entries, header says {nnz}")
    data = data.reshape(nnz, 3)
    genes, cells, vals = data[:, 0] - 1, data[:, 1] - 1, data[:, 2]
    if nnz and (genes.min() < 0 or genes.max() >= n_genes or cells.min() < 0 or cells.max() >= n_cells):
        raise ValueError(f"{path}: index out of range")
    if nnz and (vals.min() < 0 or vals.max() > 65535):
        raise ValueError(f"{path}: counts must be in [0, 65535]")
    keep = vals > 0
    genes, cells, vals = genes[keep], cells[keep], vals[keep]
    order = np.lexsort((genes, cells))
    genes, cells, vals = genes[order], cells[order], vals[order]
    if genes.size > 1 and np.any((cells[1:] == cells[:-1]) & (genes[1:] == genes[:-1])):
        raise ValueError(f"{path}: duplicate (feature, barcode) entries")
    row_ptr = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(np.bincount(cells, minlength=n_cells), out=row_ptr[1:])
    return row_ptr, genes.astype(np.int32), vals.astype(np.int32), n_genes, n_cells


def _csr(row_ptr, col, val, n_genes: int):
    rp = torch.as_tensor(row_ptr).to(device="cuda", dtype=torch.int64).contiguous()
    cl = torch.as_tensor(col).to(device="cuda", dtype=torch.int32).contiguous()
    vl = torch.as_tensor(val).to(device="cuda", dtype=torch.int32).contiguous()
    csr = C.dpmm_csr(rp.numel() - 1, int(n_genes), 0, cl.numel(), rp.data_ptr(),
                     cl.data_ptr() if cl.numel() else None, vl.data_ptr() if vl.numel() else None)
    return csr, (rp, cl, vl)


def _moments_dev(row_ptr, col, val, n_genes: int):
    csr, keep = _csr(row_ptr, col, val, n_genes)
    s = torch.zeros(n_genes, dtype=torch.int64, device="cuda")
    q = torch.zeros(n_genes, dtype=torch.int64, device="cuda")
    C.dpmm_gene_moments(csr, s.data_ptr(), q.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return s, q, keep


def gene_moments(row_ptr, col, val, n_genes: int):
    """Exact (sum_i x_iu, sum_i x_iu^2) per gene, as Python-int numpy object arrays."""
    s, q, _ = _moments_dev(row_ptr, col, val, n_genes)
    torch.cuda.current_stream().synchronize()
    # stored as uint64; both fit in int64 for valid data
    return s.cpu().numpy().astype(object), q.cpu().numpy().astype(object)


def top_genes(row_ptr, col, val, n_genes: int, k: int):
    """The k genes of largest standard deviation across the cells (Section 3),
    ranked exactly on the GPU (equal variances: the lower gene first):
    (genes in increasing order as numpy int64, the gene -> place map as a
    device tensor for filter_genes, the standard deviations as numpy)."""
    n_cells = len(row_ptr) - 1
    s, q, _ = _moments_dev(row_ptr, col, val, n_genes)
    gmap = torch.empty(n_genes, dtype=torch.int32, device="cuda")
    std = torch.empty(n_genes, dtype=torch.float64, device="cuda")
    C.dpmm_top_genes(s.data_ptr(), q.data_ptr(), n_genes, n_cells, int(k), gmap.data_ptr(), std.data_ptr(),
                     torch.cuda.current_stream().cuda_stream)
    torch.cuda.current_stream().synchronize()
    genes = np.nonzero(gmap.cpu().numpy() >= 0)[0].astype(np.int64)
    return genes, gmap, std.cpu().numpy()


def filter_genes(row_ptr, col, val, n_genes: int, genes):
    """The CSR restricted to ``genes`` (increasing gene indices, or the
    gene -> place map of top_genes as a device tensor), renumbered
    0..len-1, on the GPU: (row_ptr, col, val) as device tensors."""
    csr, keep = _csr(row_ptr, col, val, n_genes)
    if isinstance(genes, torch.Tensor) and genes.is_cuda:
        gm = genes.to(torch.int32).contiguous()
    else:
        genes = np.asarray(genes, dtype=np.int64)
        if genes.size and (np.any(np.diff(genes) <= 0) or genes[0] < 0 or genes[-1] >= n_genes):
            raise ValueError("genes must be increasing and in [0, n_genes)")
        gmap = np.full(n_genes, -1, dtype=np.int32)
        gmap[genes] = np.arange(genes.size, dtype=np.int32)
        gm = torch.from_numpy(gmap).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    rp_out = torch.empty(csr.n_cells + 1, dtype=torch.int64, device="cuda")
    nnz = C.dpmm_filter_genes(csr, gm.data_ptr(), rp_out.data_ptr(), None, None, stream)
    col_out = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    val_out = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    C.dpmm_filter_genes(csr, gm.data_ptr(), rp_out.data_ptr(), col_out.data_ptr(), val_out.data_ptr(), stream)
    torch.cuda.current_stream().synchronize()
    return rp_out, col_out[:nnz], val_out[:nnz]
