"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws test matrices; it holds none of the randomized SVD's
arithmetic (the Gaussian test matrix of the method is generated separately
by each side from its counter-based definition).  Both the tests (GPU path
and oracle) and bench.py take their inputs from here.

The paper's own inputs (two SuiteSparse matrices and a 512 x 512 image) are
not available; these matrices stand in for them with stated shapes, spectra
and noise.  Recipes:

  dense_lowrank: A = U diag(sigma) V^T + noise_std * N(0, 1), U (m x r) and
    V (n x r) Haar-distributed orthonormal columns (QR of a Gaussian matrix
    with the columns multiplied by sign(diag R), Mezzadri 2007).  "N(0, x)"
    in a recipe is read as standard deviation x.

Named recipes (sizes, spectra, seeds):
  plain_small    2000 x 1000, sigma_i = exp(-i/50) (i = 1..1000), noise 1e-6,
                 FP64, seed 1, k = 20, p = 10, q = 2
  plain_gpu      50000 x 20000, sigma_i = 1/i (i <= 2000), noise 1e-4, FP32,
                 seed 2, k = 100, p = 20, q = 2, 4096 x 4096 tiles
  mixed          65536 x 32768, sigma_i = i^-0.5, noise 1e-4, FP32, seed 5,
                 k = 128, p = 32, q = 3
  fd             256 x 128, sigma_i = i^-0.5 (i <= 128), noise 1e-4, seeds
                 100..104, k = 16, p = 112, q = 3
  ooc            200000 x 100000 (run at half scale), sigma_i = i^-0.8 (i <= 500),
                 noise 1e-5, FP32, seed 3, in pinned host memory, 16 GB HBM budget
  sparse         zipf_csr: 2e6 x 5e5, exactly 50 distinct columns per row drawn
                 Zipf(1.1) over ranks 1..n (duplicates redrawn), column =
                 perm(rank - 1) with a seeded permutation, sorted within rows,
                 values log(1 + c), c ~ Poisson(3) + 1; FP32 values, int32
                 indices, seed 4 (the paper's SuiteSparse inputs are absent)
  hamrle3_like   banded_random_coo: 1,447,360 x 1,447,360 with 5,514,242 entries,
                 the shape of the paper's first SuiteSparse test matrix (§4.1);
                 tridiagonal band (values 4 + |N(0,1)| on the diagonal, N(0,1)
                 off it) plus uniformly placed N(0,1) entries, seed 6
  circuit5m_like banded_random_coo: 5,558,326 x 5,558,326 with 59,524,291
                 entries (the second matrix's shape), band of half-width 2, seed 7
  The structure of the real matrices is not known here: these stand-ins keep
  only their order and entry counts.
Scaled-down variants keep the spectrum law and noise and shrink m, n.
"""

import math

import numpy as np
import torch


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def haar_columns(rows, cols, gen, device="cpu", dtype=torch.float64):
    """rows x cols matrix with Haar-distributed orthonormal columns."""
    G = torch.randn(rows, cols, generator=gen, device=device, dtype=dtype)
    Qm, R = torch.linalg.qr(G, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1
    return Qm * d[None, :]


def dense_lowrank(m, n, sigma, noise_std, seed, device="cpu", out_dtype=torch.float32,
                  work_dtype=torch.float64):
    """A = U diag(sigma) V^T + noise_std * N(0,1) as an (m, n) torch tensor
    (row-major) of out_dtype on `device`."""
    sigma = torch.as_tensor(np.asarray(sigma, dtype=np.float64), dtype=work_dtype, device=device)
    r = int(sigma.numel())
    if r > min(m, n):
        raise ValueError("rank exceeds min(m, n)")
    g = _gen(seed, device)
    U = haar_columns(m, r, g, device, work_dtype)
    V = haar_columns(n, r, g, device, work_dtype)
    A = (U * sigma[None, :]) @ V.T
    del U, V
    if noise_std:
        A.add_(torch.randn(m, n, generator=g, device=device, dtype=work_dtype), alpha=float(noise_std))
    return A.to(out_dtype)


def spectrum_exp(count, scale=50.0):
    i = np.arange(1, count + 1, dtype=np.float64)
    return np.exp(-i / scale)


def spectrum_pow(count, power):
    i = np.arange(1, count + 1, dtype=np.float64)
    return i ** (-float(power))


RECIPES = {
    "plain_small": dict(m=2000, n=1000, spectrum=("exp", 1000, 50.0), noise=1e-6, seed=1,
                        k=20, p=10, q=2, dtype="f64", tile=(2000, 1000)),
    "plain_gpu": dict(m=50000, n=20000, spectrum=("pow", 2000, 1.0), noise=1e-4, seed=2,
                      k=100, p=20, q=2, dtype="f32", tile=(4096, 4096)),
    "mixed": dict(m=65536, n=32768, spectrum=("pow", 32768, 0.5), noise=1e-4, seed=5,
                  k=128, p=32, q=3, dtype="f32", tile=(4096, 4096)),
    # out-of-core: A lives in pinned host memory, HBM budget 16 GB
    "ooc": dict(m=200000, n=100000, spectrum=("pow", 500, 0.8), noise=1e-5, seed=3,
                k=200, p=30, q=2, dtype="f32", tile=(8192, 8192)),
}


def recipe_sigma(spec):
    kind = spec[0]
    if kind == "exp":
        return spectrum_exp(spec[1], spec[2])
    if kind == "pow":
        return spectrum_pow(spec[1], spec[2])
    raise ValueError(kind)


def make(name, device="cpu", scale=1.0, out_dtype=None):
    """Build a named recipe (optionally with m, n and the spectrum length
    scaled by `scale`).  Returns (A, meta)."""
    r = dict(RECIPES[name])
    m = max(8, int(round(r["m"] * scale)))
    n = max(8, int(round(r["n"] * scale)))
    spec = r["spectrum"]
    cnt = min(max(1, int(round(spec[1] * scale))), m, n)
    sigma = recipe_sigma((spec[0], cnt) + tuple(spec[2:]))
    if out_dtype is None:
        out_dtype = torch.float64 if r["dtype"] == "f64" else torch.float32
    A = dense_lowrank(m, n, sigma, r["noise"], r["seed"], device=device, out_dtype=out_dtype)
    meta = dict(r, m=m, n=n, sigma=sigma, scale=scale)
    return A, meta


def zipf_csr(m, n, per_row, s=1.1, seed=4, device="cpu", draws=None):
    """CSR (rowptr int32 [m + 1], colind int32 [nnz], values float32 [nnz])
    with exactly per_row distinct columns in every row; see the module
    docstring for the distribution."""
    g = _gen(seed, device)
    draws = draws or max(2 * per_row, per_row + 64)
    ranks = torch.arange(1, n + 1, device=device, dtype=torch.float64)
    cdf = torch.cumsum(ranks ** (-float(s)), 0)
    cdf /= cdf[-1].clone()
    perm = torch.randperm(n, generator=g, device=device)
    cols = torch.empty(m, per_row, dtype=torch.int64, device=device)
    todo = torch.arange(m, device=device)
    while todo.numel():
        u = torch.rand(todo.numel(), draws, generator=g, device=device, dtype=torch.float64)
        r = torch.searchsorted(cdf, u).clamp_(max=n - 1)          # rank - 1
        srt, order = torch.sort(r, dim=1, stable=True)
        first = torch.ones_like(srt, dtype=torch.bool)
        first[:, 1:] = srt[:, 1:] != srt[:, :-1]
        # keep the first occurrence of each rank, in draw order
        pos = torch.where(first, order, torch.full_like(order, draws))
        pos_sorted, _ = torch.sort(pos, dim=1)
        ok = pos_sorted[:, per_row - 1] < draws
        keep = pos_sorted[ok][:, :per_row]
        picked = torch.gather(r[ok], 1, keep)
        cols[todo[ok]] = perm[picked]
        todo = todo[~ok]
    cols, _ = torch.sort(cols, dim=1)
    c = torch.poisson(torch.full((m, per_row), 3.0, device=device, dtype=torch.float64),
                      generator=g) + 1.0
    values = torch.log1p(c).to(torch.float32).reshape(-1)
    rowptr = (torch.arange(m + 1, device=device, dtype=torch.int64) * per_row).to(torch.int32)
    return rowptr, cols.reshape(-1).to(torch.int32), values


def banded_random_coo(n, nnz, half_width, seed, device="cpu", index_dtype=torch.int64):
    """Square n x n COO (rowind, colind, values float32) with exactly nnz
    entries: the band |i - j| <= half_width (clipped at the edges), then
    uniformly placed entries up to nnz (a repeated (i, j) adds up).  Band
    values: 4 + |N(0,1)| on the diagonal, N(0,1) off it; others N(0,1).
    Entries come in band-then-random order (not sorted by row)."""
    g = _gen(seed, device)
    rows, cols = [], []
    for d in range(-half_width, half_width + 1):
        i = torch.arange(max(0, -d), min(n, n - d), device=device, dtype=torch.int64)
        rows.append(i)
        cols.append(i + d)
    r = torch.cat(rows)
    c = torch.cat(cols)
    nb = int(r.numel())
    if nb > nnz:
        raise ValueError("nnz is smaller than the band")
    extra = nnz - nb
    r = torch.cat([r, torch.randint(0, n, (extra,), generator=g, device=device)])
    c = torch.cat([c, torch.randint(0, n, (extra,), generator=g, device=device)])
    v = torch.randn(nnz, generator=g, device=device, dtype=torch.float32)
    diag = torch.zeros(nnz, dtype=torch.bool, device=device)
    diag[:nb] = r[:nb] == c[:nb]
    v = torch.where(diag, 4.0 + v.abs(), v)
    return r.to(index_dtype), c.to(index_dtype), v


SPARSE_STANDINS = {
    "hamrle3_like": dict(n=1447360, nnz=5514242, half_width=1, seed=6),
    "circuit5m_like": dict(n=5558326, nnz=59524291, half_width=2, seed=7),
}


def fd_instance(seed, m=256, n=128, noise=1e-4, device="cpu"):
    sigma = spectrum_pow(min(m, n), 0.5)
    return dense_lowrank(m, n, sigma, noise, seed, device=device, out_dtype=torch.float64)


def sizes_ok(m, n, k, p):
    return k >= 1 and p >= 0 and k + p <= min(m, n)


def ceil_div(a, b):
    return -(-a // b)


__all__ = ["dense_lowrank", "haar_columns", "make", "fd_instance", "zipf_csr",
           "banded_random_coo", "SPARSE_STANDINS",
           "RECIPES", "recipe_sigma", "spectrum_exp", "spectrum_pow", "math"]
