"""Python binding of the randomized SVD library (argument marshalling only).

PyTorch supplies device memory and the stream; every step of the computation
runs in the HIP kernels of librsvd.so.  Panels handed to and from the library
are column-major: a torch tensor of shape (rows, cols) with strides
(1, ld), built as ``torch.empty(cols, ld)[:, :rows].T``.
"""

import ctypes

import torch

from . import _lib as L

_DT = {torch.float32: L.F32, torch.float64: L.F64, torch.bfloat16: L.BF16}
_PREC = {"fp32": L.F32, "bf16": L.BF16, "fp8": L.FP8E4M3}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def col_major(rows, cols, dtype=torch.float32, device="cuda", ld=None):
    """Empty column-major (rows, cols) tensor with leading dimension ld."""
    ld = rows if ld is None else ld
    return torch.empty(cols, ld, dtype=dtype, device=device)[:, :rows].T


def _ld_col_major(t):
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("panel must be column-major (stride (1, ld))")
    return t.stride(1) if t.shape[1] > 1 else max(t.shape[0], 1)


def _ld_row_major(A):
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be row-major with unit column stride")
    return A.stride(0) if A.shape[0] > 1 else A.shape[1]


def _csr_arrays(rowptr, colind, values, plan):
    if plan.nnz is None:
        raise ValueError("the plan is for dense input")
    rowptr = rowptr.to(torch.int32).contiguous()
    colind = colind.to(torch.int32).contiguous()
    values = values.to(torch.float32).contiguous()
    if rowptr.numel() != plan.m + 1 or colind.numel() != plan.nnz or values.numel() != plan.nnz:
        raise ValueError("CSR arrays do not match the plan")
    if not (rowptr.is_cuda and colind.is_cuda and values.is_cuda):
        raise ValueError("CSR arrays must be cuda tensors")
    return rowptr, colind, values


class Checkpoint:
    """State of a factorisation after a completed pass over A (header fields
    as in rsvd_checkpoint, plus the FP32 panel as a (rows, cols) column-major
    numpy array).  Files hold the header's bytes followed by the panel's."""

    def __init__(self, header, panel):
        self.header = header          # L.Checkpoint
        self.panel = panel            # numpy float32, shape (cols, rows) C-order = column-major

    @property
    def passes(self):
        return self.header.passes

    def save(self, path):
        import numpy as np
        with open(path, "wb") as f:
            f.write(bytes(self.header))
            f.write(np.ascontiguousarray(self.panel, dtype=np.float32).tobytes())

    @classmethod
    def load(cls, path):
        import numpy as np
        with open(path, "rb") as f:
            raw = f.read(ctypes.sizeof(L.Checkpoint))
            if len(raw) != ctypes.sizeof(L.Checkpoint):
                raise ValueError("truncated checkpoint header")
            hdr = L.Checkpoint.from_buffer_copy(raw)
            if hdr.magic != L.CKPT_MAGIC:
                raise ValueError("not a checkpoint file")
            count = int(hdr.rows) * int(hdr.cols)
            panel = np.fromfile(f, dtype=np.float32, count=count)
        if panel.size != count:
            raise ValueError("truncated checkpoint panel")
        return cls(hdr, panel.reshape(int(hdr.cols), int(hdr.rows)))


class Plan:
    """A validated problem with its tile map and workspace size."""

    def __init__(self, m, n, k, p, q, seed=0, dtype=torch.float32, precision="fp32",
                 tile=None, grid=(1, 1), hbm_budget=0, flags=0, backward=False, host=False,
                 nnz=None, auto_q=False, q_tol=0.0, coo=False, a_budget=0, new_budget=0):
        """host=True: A stays in pinned host memory and is streamed to the
        device tile by tile on every pass (hbm_budget bounds the slots).
        a_budget / new_budget: device bytes for the tiles of A and for the
        matrices the plan builds (Section 3.5's per-matrix and new-matrix
        limits; 0 takes the next limit, new_budget then hbm_budget).  A
        host-resident A whose a_budget holds every tile is copied once per
        call and kept resident for the later passes.
        nnz: A is sparse (CSR with int32 indices, FP32 values) with nnz
        nonzeros; use factor_csr / factor with a sparse CSR tensor.  With
        coo=True the nnz entries come as COO arrays (factor_coo).
        auto_q: q is a maximum; the power iteration stops once the leading k
        singular values change by at most q_tol (relative) from one q to the
        next (Section 2.2); info["q_used"] reports the q chosen."""
        if backward:
            flags |= L.FLAG_BACKWARD
        if auto_q:
            flags |= L.FLAG_AUTO_Q
        prob = L.Problem(m=m, n=n, k=k, p=p, q=q, format=L.DENSE if nnz is None else (L.COO if coo else L.CSR),
                         dtype=_DT.get(dtype, -99),
                         loc=L.LOC_HOST_PINNED if host else L.LOC_DEVICE, reserved=0, seed=seed,
                         nnz=0 if nnz is None else int(nnz))
        # one precision for every pass, or (sketch, power, project)
        names = (precision,) * 3 if isinstance(precision, str) else tuple(precision)
        if len(names) != 3:
            raise ValueError("precision: a name or a (sketch, power, project) triple")
        ps, pw, pj = (_PREC.get(x, -99) for x in names)
        tm, tn = (tile if tile is not None else (0, 0))
        opt = L.Options(prec_sketch=ps, prec_power=pw, prec_project=pj, ortho=L.ORTHO_EACH,
                        tile_m=tm, tile_n=tn, grid_p=grid[0], grid_q=grid[1],
                        hbm_budget_bytes=int(hbm_budget), flags=flags, reserved=0,
                        q_tol=float(q_tol), a_budget_bytes=int(a_budget),
                        new_budget_bytes=int(new_budget))
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        st = L.lib().rsvd_plan(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(h),
                               ctypes.byref(ws))
        L.check(st, None)
        self.handle = h
        self.ws_bytes = ws.value
        self.m, self.n, self.k, self.p, self.q, self.seed = m, n, k, p, q, seed
        self.l = k + p
        self.dtype = dtype
        self.host = host
        self.nnz = nnz
        self.coo = coo

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                L.lib().rsvd_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def set_streams(self, copy_stream=None, side_stream=None):
        """rsvd_plan_set_streams: caller-owned torch streams for the tile
        copies (host-resident A) and the deferred CholeskyQR passes; None lets
        the plan create its own.  The streams must outlive their use."""
        cs = ctypes.c_void_p(copy_stream.cuda_stream) if copy_stream is not None else None
        ss = ctypes.c_void_p(side_stream.cuda_stream) if side_stream is not None else None
        L.check(L.lib().rsvd_plan_set_streams(self.handle, cs, ss), self.handle)
        self._streams = (copy_stream, side_stream)

    def workspace(self, device="cuda"):
        return torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)

    def tile_map(self):
        n = ctypes.c_size_t()
        L.check(L.lib().rsvd_tile_map(self.handle, None, 0, ctypes.byref(n)), self.handle)
        buf = (ctypes.c_int64 * n.value)()
        L.check(L.lib().rsvd_tile_map(self.handle, buf, n.value, ctypes.byref(n)), self.handle)
        return torch.tensor(list(buf), dtype=torch.int64).reshape(-1, 12)

    def visit_order(self, pass_index):
        n = ctypes.c_size_t()
        L.check(L.lib().rsvd_visit_order(self.handle, pass_index, None, 0, ctypes.byref(n)),
                self.handle)
        buf = (ctypes.c_int64 * n.value)()
        L.check(L.lib().rsvd_visit_order(self.handle, pass_index, buf, n.value, ctypes.byref(n)),
                self.handle)
        return torch.tensor(list(buf), dtype=torch.int64)

    # ---- calls that run on the GPU ---------------------------------------
    def factor(self, A, ws=None, out=None, stream=None, report=True):
        """Randomized SVD of A (cuda tensor, row-major).  Returns
        (U (m x k, column-major), S (k, FP64), V (n x k, column-major), info)."""
        lda = _ld_row_major(A)
        if A.dtype != self.dtype or tuple(A.shape) != (self.m, self.n):
            raise ValueError("A does not match the plan")
        if self.host != (not A.is_cuda):
            raise ValueError("A must be a pinned CPU tensor for a host plan, a cuda tensor otherwise")
        dev = torch.device("cuda", torch.cuda.current_device()) if self.host else A.device
        ws = self.workspace(dev) if ws is None else ws
        if out is None:
            U = col_major(self.m, self.k, device=dev)
            S = torch.empty(self.k, dtype=torch.float64, device=dev)
            V = col_major(self.n, self.k, device=dev)
        else:
            U, S, V = out
        rep = L.Report() if report else None
        st = L.lib().rsvd_factor(self.handle, _ptr(A), lda, _ptr(ws), _ptr(U), _ld_col_major(U),
                                 _ptr(S), _ptr(V), _ld_col_major(V), _stream_ptr(stream),
                                 ctypes.byref(rep) if rep is not None else None)
        L.check(st, self.handle)
        info = {"status": st}
        if rep is not None:
            info.update(stage_ms=list(rep.stage_ms), total_ms=rep.total_ms,
                        flops_alg=rep.flops_alg, bytes_alg=rep.bytes_alg,
                        gemm_nn_ms=rep.gemm_nn_ms, gemm_tn_ms=rep.gemm_tn_ms,
                        gemm_nn_launches=rep.gemm_nn_launches,
                        gemm_tn_launches=rep.gemm_tn_launches,
                        ws_bytes=rep.ws_bytes, dropped=rep.dropped,
                        jacobi_sweeps=rep.jacobi_sweeps, nonfinite=rep.nonfinite,
                        slots=rep.slots, h2d_bytes=rep.h2d_bytes, tile_loads=rep.tile_loads,
                        q_used=rep.q_used, q_delta=rep.q_delta, sketch_ms=rep.sketch_ms,
                        peak_hbm=rep.peak_hbm)
        return U, S, V, info

    def factor_noalloc(self, A, out=None, stream=None):
        """rsvd_factor_noalloc: the library's static device workspace instead of
        a caller buffer (dense A in device memory).  Returns (U, S, V, status);
        no report."""
        lda = _ld_row_major(A)
        if A.dtype != self.dtype or tuple(A.shape) != (self.m, self.n) or not A.is_cuda:
            raise ValueError("A must be a cuda tensor that matches the plan")
        if out is None:
            U = col_major(self.m, self.k, device=A.device)
            S = torch.empty(self.k, dtype=torch.float64, device=A.device)
            V = col_major(self.n, self.k, device=A.device)
        else:
            U, S, V = out
        st = L.lib().rsvd_factor_noalloc(self.handle, _ptr(A), lda, _ptr(U), _ld_col_major(U),
                                         _ptr(S), _ptr(V), _ld_col_major(V), _stream_ptr(stream))
        L.check(st, self.handle)
        return U, S, V, st

    def factor_resumable(self, A, stop_after=0, resume=None, save=True, ws=None, stream=None,
                         report=True):
        """rsvd_factor_resumable: returns (U, S, V, info, ckpt).  ``stop_after``
        (1 .. 2q + 2) ends the call after that pass (U, S, V are then None);
        ``resume`` is a Checkpoint to continue from; with ``save`` the returned
        ckpt holds the state after the last completed pass."""
        import numpy as np
        lda = _ld_row_major(A)
        if A.dtype != self.dtype or tuple(A.shape) != (self.m, self.n):
            raise ValueError("A does not match the plan")
        if self.host != (not A.is_cuda):
            raise ValueError("A must be a pinned CPU tensor for a host plan, a cuda tensor otherwise")
        dev = torch.device("cuda", torch.cuda.current_device()) if self.host else A.device
        ws = self.workspace(dev) if ws is None else ws
        U = col_major(self.m, self.k, device=dev)
        S = torch.empty(self.k, dtype=torch.float64, device=dev)
        V = col_major(self.n, self.k, device=dev)
        nbytes = ctypes.c_size_t()
        L.check(L.lib().rsvd_checkpoint_bytes(self.handle, ctypes.byref(nbytes)), self.handle)
        out_hdr = L.Checkpoint() if save else None
        out_panel = np.zeros(nbytes.value // 4, dtype=np.float32) if save else None
        in_hdr, in_panel = None, None
        if resume is not None:
            in_hdr = resume.header
            in_panel = np.ascontiguousarray(resume.panel, dtype=np.float32)
        rep = L.Report() if report else None
        st = L.lib().rsvd_factor_resumable(
            self.handle, _ptr(A), lda, _ptr(ws), _ptr(U), _ld_col_major(U), _ptr(S), _ptr(V),
            _ld_col_major(V), _stream_ptr(stream),
            ctypes.byref(rep) if rep is not None else None,
            ctypes.byref(in_hdr) if in_hdr is not None else None,
            ctypes.c_void_p(in_panel.ctypes.data) if in_panel is not None else None,
            int(stop_after),
            ctypes.byref(out_hdr) if out_hdr is not None else None,
            ctypes.c_void_p(out_panel.ctypes.data) if out_panel is not None else None)
        L.check(st, self.handle)
        ckpt = None
        if save and out_hdr.magic == L.CKPT_MAGIC:
            rows, cols = int(out_hdr.rows), int(out_hdr.cols)
            ckpt = Checkpoint(out_hdr, out_panel[:rows * cols].reshape(cols, rows).copy())
        info = {"status": st}
        if st == L.STOPPED:
            return None, None, None, info, ckpt
        if rep is not None:
            info.update(stage_ms=list(rep.stage_ms), total_ms=rep.total_ms,
                        dropped=rep.dropped, jacobi_sweeps=rep.jacobi_sweeps)
        return U, S, V, info, ckpt

    def backward(self, A, gU=None, gS=None, gV=None, ws=None, stream=None, report=True):
        """gA (m x n, row-major FP32) of the truncated-SVD adjoint; the plan must
        have been made with backward=True.  Cotangents may be None (zero)."""
        lda = _ld_row_major(A)
        ws = self.workspace(A.device) if ws is None else ws
        gA = torch.empty(self.m, self.n, dtype=torch.float32, device=A.device)

        def panel(g, rows):
            if g is None:
                return None, 0
            g = g.to(torch.float32)
            if g.dim() != 2 or g.shape != (rows, self.k):
                raise ValueError("cotangent shape mismatch")
            if g.stride(0) != 1:
                g = g.T.contiguous().T            # column-major copy
            return g, _ld_col_major(g)

        gUc, ldgu = panel(gU, self.m)
        gVc, ldgv = panel(gV, self.n)
        gSc = None if gS is None else gS.to(torch.float64).contiguous()
        rep = L.Report() if report else None
        st = L.lib().rsvd_backward(self.handle, _ptr(A), lda, _ptr(gUc), ldgu, _ptr(gSc), _ptr(gVc),
                                   ldgv, _ptr(gA), gA.stride(0), _ptr(ws), _stream_ptr(stream),
                                   ctypes.byref(rep) if rep is not None else None)
        L.check(st, self.handle)
        return gA, {"status": st, "total_ms": rep.total_ms if rep is not None else None}

    def residual(self, A, U, S, V, ws=None, stream=None):
        """||A - U diag(S) V^T||_F computed on the device (FP64 sums)."""
        ws = self.workspace(A.device) if ws is None else ws
        out = torch.empty(1, dtype=torch.float64, device=A.device)
        st = L.lib().rsvd_residual(self.handle, _ptr(A), _ld_row_major(A), _ptr(U), _ld_col_major(U),
                                   _ptr(S), _ptr(V), _ld_col_major(V), _ptr(out), _ptr(ws),
                                   _stream_ptr(stream))
        L.check(st, self.handle)
        return out

    def factor_csr(self, rowptr, colind, values, ws=None, out=None, stream=None, report=True):
        """Randomized SVD of a sparse A given as CSR device arrays (int32
        rowptr[m + 1], int32 colind[nnz], float32 values[nnz])."""
        rowptr, colind, values = _csr_arrays(rowptr, colind, values, self)
        dev = rowptr.device
        ws = self.workspace(dev) if ws is None else ws
        if out is None:
            U = col_major(self.m, self.k, device=dev)
            S = torch.empty(self.k, dtype=torch.float64, device=dev)
            V = col_major(self.n, self.k, device=dev)
        else:
            U, S, V = out
        rep = L.Report() if report else None
        st = L.lib().rsvd_factor_csr(self.handle, _ptr(rowptr), _ptr(colind), _ptr(values), _ptr(ws),
                                     _ptr(U), _ld_col_major(U), _ptr(S), _ptr(V), _ld_col_major(V),
                                     _stream_ptr(stream),
                                     ctypes.byref(rep) if rep is not None else None)
        L.check(st, self.handle)
        info = {"status": st}
        if rep is not None:
            info.update(stage_ms=list(rep.stage_ms), total_ms=rep.total_ms,
                        flops_alg=rep.flops_alg, bytes_alg=rep.bytes_alg,
                        gemm_nn_ms=rep.gemm_nn_ms, gemm_tn_ms=rep.gemm_tn_ms,
                        gemm_nn_launches=rep.gemm_nn_launches,
                        gemm_tn_launches=rep.gemm_tn_launches, ws_bytes=rep.ws_bytes,
                        dropped=rep.dropped, jacobi_sweeps=rep.jacobi_sweeps,
                        q_used=rep.q_used, q_delta=rep.q_delta, peak_hbm=rep.peak_hbm)
        return U, S, V, info

    def factor_coo(self, rowind, colind, values, ws=None, out=None, stream=None, report=True):
        """Randomized SVD of a sparse A given as COO device arrays (rowind and
        colind both int32 or both int64, nnz entries in any order; float32
        values).  Returns (U, S, V, info) as factor_csr."""
        if not self.coo:
            raise ValueError("the plan is not for COO input (Plan(..., nnz=, coo=True))")
        if rowind.dtype != colind.dtype or rowind.dtype not in (torch.int32, torch.int64):
            raise ValueError("COO indices must both be int32 or both int64")
        rowind, colind = rowind.contiguous(), colind.contiguous()
        values = values.to(torch.float32).contiguous()
        if rowind.numel() != self.nnz or colind.numel() != self.nnz or values.numel() != self.nnz:
            raise ValueError("COO arrays do not match the plan")
        if not (rowind.is_cuda and colind.is_cuda and values.is_cuda):
            raise ValueError("COO arrays must be cuda tensors")
        bits = 64 if rowind.dtype == torch.int64 else 32
        dev = rowind.device
        ws = self.workspace(dev) if ws is None else ws
        if out is None:
            U = col_major(self.m, self.k, device=dev)
            S = torch.empty(self.k, dtype=torch.float64, device=dev)
            V = col_major(self.n, self.k, device=dev)
        else:
            U, S, V = out
        rep = L.Report() if report else None
        st = L.lib().rsvd_factor_coo(self.handle, _ptr(rowind), _ptr(colind), bits, _ptr(values),
                                     _ptr(ws), _ptr(U), _ld_col_major(U), _ptr(S), _ptr(V),
                                     _ld_col_major(V), _stream_ptr(stream),
                                     ctypes.byref(rep) if rep is not None else None)
        L.check(st, self.handle)
        info = {"status": st}
        if rep is not None:
            info.update(stage_ms=list(rep.stage_ms), total_ms=rep.total_ms,
                        flops_alg=rep.flops_alg, bytes_alg=rep.bytes_alg,
                        gemm_nn_ms=rep.gemm_nn_ms, gemm_tn_ms=rep.gemm_tn_ms,
                        gemm_nn_launches=rep.gemm_nn_launches,
                        gemm_tn_launches=rep.gemm_tn_launches, ws_bytes=rep.ws_bytes,
                        dropped=rep.dropped, jacobi_sweeps=rep.jacobi_sweeps,
                        peak_hbm=rep.peak_hbm)
        return U, S, V, info

    def step_spmm(self, op, rowptr, colind, values, X, ws=None, stream=None):
        rowptr, colind, values = _csr_arrays(rowptr, colind, values, self)
        rows_out = self.m if op == 0 else self.n
        out = col_major(rows_out, self.l, device=X.device)
        ws = self.workspace(X.device) if ws is None else ws
        st = L.lib().rsvd_step_spmm(self.handle, op, _ptr(rowptr), _ptr(colind), _ptr(values),
                                    _ptr(X), _ld_col_major(X), _ptr(out), _ld_col_major(out),
                                    _ptr(ws), _stream_ptr(stream))
        L.check(st, self.handle)
        return out

    def step_product(self, op, A, X, ws=None, stream=None):
        rows_out = self.m if op == 0 else self.n
        out = col_major(rows_out, self.l, device=A.device)
        ws = self.workspace(A.device) if ws is None else ws
        st = L.lib().rsvd_step_product(self.handle, op, _ptr(A), _ld_row_major(A), _ptr(X),
                                       _ld_col_major(X), _ptr(out), _ld_col_major(out), _ptr(ws),
                                       _stream_ptr(stream))
        L.check(st, self.handle)
        return out

    def step_orth(self, side, Y, ws=None, stream=None):
        rows = self.m if side == 0 else self.n
        Q = col_major(rows, self.l, device=Y.device)
        ws = self.workspace(Y.device) if ws is None else ws
        st = L.lib().rsvd_step_orth(self.handle, side, _ptr(Y), _ld_col_major(Y), _ptr(Q),
                                    _ld_col_major(Q), _ptr(ws), _stream_ptr(stream))
        L.check(st, self.handle)
        return Q

    def step_gram(self, side, Y, ws=None, stream=None):
        G = torch.empty(self.l, self.l, dtype=torch.float64, device=Y.device)
        ws = self.workspace(Y.device) if ws is None else ws
        st = L.lib().rsvd_step_gram(self.handle, side, _ptr(Y), _ld_col_major(Y), _ptr(G),
                                    _ptr(ws), _stream_ptr(stream))
        L.check(st, self.handle)
        return G

    def step_small_svd(self, Bt, ws=None, stream=None):
        sig = torch.empty(self.l, dtype=torch.float64, device=Bt.device)
        ub = torch.empty(self.l, self.l, dtype=torch.float64, device=Bt.device)
        ws = self.workspace(Bt.device) if ws is None else ws
        st = L.lib().rsvd_step_small_svd(self.handle, _ptr(Bt), _ld_col_major(Bt), _ptr(sig),
                                         _ptr(ub), _ptr(ws), _stream_ptr(stream))
        L.check(st, self.handle)
        return sig, ub


def factor(A, k, p, q, seed=0, precision="fp32", tile=None, flags=0, stream=None,
           hbm_budget=0):
    """One-call randomized SVD: returns (U, S, V, info).  A pinned CPU tensor
    is streamed from host memory (out of core); a cuda tensor is used in place;
    a sparse CSR cuda tensor runs the sparse products."""
    if A.layout == torch.sparse_csr:
        plan = Plan(A.shape[0], A.shape[1], k, p, q, seed=seed, flags=flags, nnz=A._nnz())
        return plan.factor_csr(A.crow_indices(), A.col_indices(), A.values(), stream=stream)
    plan = Plan(A.shape[0], A.shape[1], k, p, q, seed=seed, dtype=A.dtype, precision=precision,
                tile=tile, flags=flags, hbm_budget=hbm_budget, host=not A.is_cuda)
    return plan.factor(A, stream=stream)


class RSVD(torch.autograd.Function):
    """Differentiable randomized SVD: forward rsvd_factor, backward
    rsvd_backward (the range basis is recomputed from the seed).

        U, S, V = RSVD.apply(A, k, p, q, seed, precision)
    """

    @staticmethod
    def forward(ctx, A, k, p, q, seed=0, precision="fp32"):
        plan = Plan(A.shape[0], A.shape[1], k, p, q, seed=seed, dtype=A.dtype,
                    precision=precision, backward=True)
        U, S, V, _ = plan.factor(A.detach())
        ctx.plan = plan
        ctx.save_for_backward(A.detach())
        return U, S, V

    @staticmethod
    def backward(ctx, gU, gS, gV):
        (A,) = ctx.saved_tensors
        gA, _ = ctx.plan.backward(A, gU, gS, gV)
        return gA.to(A.dtype), None, None, None, None, None


def philox_raw(seed, stream_id, row0, rows, blocks, device="cuda"):
    out = torch.empty(rows * blocks * 4, dtype=torch.int32, device=device)
    st = L.lib().rsvd_philox_raw(seed, stream_id, row0, rows, blocks, _ptr(out), _stream_ptr())
    L.check(st)
    return out.view(rows, blocks, 4)


def omega(seed, n, l, row0=0, rows=None, dtype=torch.float64, device="cuda"):
    rows = n - row0 if rows is None else rows
    out = torch.empty(rows, l, dtype=dtype, device=device)
    st = L.lib().rsvd_omega(seed, n, l, row0, rows, _DT[dtype], _ptr(out), l, _stream_ptr())
    L.check(st)
    return out
