"""Shared helpers of the GPU tests: run the HIP path through the C-ABI and
compare with the CPU reference."""
import numpy as np

from oracle import oracle as orc


def lib():
    from paper_1910_04796_amd import bsmm
    return bsmm


def set_path(path="auto", kernel="plain", chunk=0):
    b = lib()
    b.bsmm_set_option("path", path)
    b.bsmm_set_option("stack_kernel", kernel)
    b.bsmm_set_option("stack_chunk", str(chunk))


def gpu_multiply(alpha, A, B, beta, Cin=None, eps=0.0, path="auto", kernel="plain", chunk=0,
                 repeat=1):
    """Runs C <- filter(beta*C + alpha*A*B) on the GPU; returns the host copy
    of C and the stats of the last call."""
    b = lib()
    set_path(path, kernel, chunk)
    try:
        MA = b.Matrix.from_blocks(A)
        MB = b.Matrix.from_blocks(B)
        MC = b.Matrix.from_blocks(Cin) if Cin is not None else b.Matrix.empty(A.rbs, B.cbs)
        for _ in range(repeat):
            b.multiply(alpha, MA, MB, beta, MC, eps)
        st = b.bsmm_last_stats()
        out = MC.to_host()
        for M in (MA, MB, MC):
            M.close()
    finally:
        set_path()
    return out, st


def same_pattern(X, R):
    return (np.array_equal(np.asarray(X.row_ptr), np.asarray(R.row_ptr))
            and np.array_equal(np.asarray(X.col_ind), np.asarray(R.col_ind)))


def check_against_oracle(X, R, tol):
    """Same pattern, then relative Frobenius error of the data <= tol."""
    assert same_pattern(X, R), "block patterns differ"
    assert len(X.data) == len(R.data)
    if tol == 0.0:
        xd, rd = np.asarray(X.data), np.asarray(R.data)
        bad = np.nonzero(~((xd == rd) | (np.isnan(xd) & np.isnan(rd))))[0]
        assert len(bad) == 0, (f"not bit-exact at {len(bad)} of {len(rd)} elements, first "
                               f"{bad[:8].tolist()}: got {xd[bad[:8]].tolist()} want {rd[bad[:8]].tolist()}")
        return 0.0
    err = orc.rel_err(np.asarray(X.data), np.asarray(R.data))
    assert err <= tol, f"relative error {err:.3e} > {tol:.1e}"
    return err


def from_dense(D, rbs, cbs):
    """Block-CSR (every block stored) of a dense matrix: blocks in CSR order,
    column-major inside a block."""
    from synth import BlockCSR, pattern_full
    rbs = np.asarray(rbs, np.int32)
    cbs = np.asarray(cbs, np.int32)
    ro = np.concatenate([[0], np.cumsum(rbs)])
    co = np.concatenate([[0], np.cumsum(cbs)])
    rp, ci = pattern_full(len(rbs), len(cbs))
    data = [np.asarray(D[ro[i]:ro[i + 1], co[j]:co[j + 1]], np.float64).ravel(order="F")
            for i in range(len(rbs)) for j in range(len(cbs))]
    return BlockCSR(rbs, cbs, rp, ci, np.concatenate(data))


def device_rows(M, r0, r1):
    """Block rows [r0, r1) of a device matrix as a host block-CSR; the data
    pass through a device buffer so that only those rows reach the host."""
    import torch

    from synth import BlockCSR, block_elems
    b = lib()
    nbr, nbc, nnzb, ne = M.info()
    tdt = torch.float32 if getattr(M, "dtype", "f64") == "f32" else torch.float64
    dev = torch.empty(max(ne, 1), dtype=tdt, device="cuda")
    rp, ci, _ = b.bsmm_copy_out(M.handle, device_out=dev)
    sizes = block_elems(M.rbs, M.cbs, rp, ci)
    start = np.concatenate([[0], np.cumsum(sizes)])
    a0, a1 = int(rp[r0]), int(rp[r1])
    data = dev[int(start[a0]):int(start[a1])].cpu().numpy().astype(np.float64)
    return BlockCSR(np.asarray(M.rbs[r0:r1], np.int32), np.asarray(M.cbs, np.int32),
                    rp[r0:r1 + 1] - rp[r0], ci[a0:a1].astype(np.int32), data)
