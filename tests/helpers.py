"""Small test helpers: build problems from dense matrices, seeded inputs."""
import numpy as np

from paper_2509_20012_amd import phantom as ph


def from_dense(D, L, c=ph.C_DL, **problem):
    """Phantom from dense FP32 matrices (zeros are structural)."""
    D = np.asarray(D, np.float32)
    L = np.asarray(L, np.float32)
    R, C = D.shape
    mask = (D != 0) | (L != 0)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(R + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=R), out=row_ptr[1:])
    p = ph._empty_problem(R)
    for k, v in problem.items():
        p[k] = np.asarray(v, dtype=p[k].dtype)
    return ph.Phantom(name="dense", n_rows=R, n_cols=C, row_ptr=row_ptr,
                      col_idx=cols.astype(np.int32), d_val=D[rows, cols],
                      l_val=L[rows, cols], x0=np.ones(C, np.float32), c=c,
                      roi={"all": np.arange(R)}, **p)


def dense(pht):
    """Dense FP64 copies of D and L."""
    R, C = pht.n_rows, pht.n_cols
    D = np.zeros((R, C))
    L = np.zeros((R, C))
    rows = np.repeat(np.arange(R), np.diff(pht.row_ptr))
    D[rows, pht.col_idx] = pht.d_val
    L[rows, pht.col_idx] = pht.l_val
    return D, L


def load_filled(fo, phantom, fill, storage=0, reserve=0):
    """(Plan, DeviceProblem, x0) with the phantom's matrices loaded through the C ABI
    into a workspace whose bytes all start as `fill` (0xFF makes every float and
    double in it a NaN)."""
    import ctypes as ct
    import torch
    rp = np.ascontiguousarray(phantom.row_ptr, np.int64)
    arrays = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
              for a in (rp, phantom.col_idx.astype(np.int32), phantom.d_val.astype(np.float32),
                        phantom.l_val.astype(np.float32))]
    nbytes = fo.workspace_bytes_csr(rp, phantom.n_cols, storage, 0, reserve)
    ws = torch.full((nbytes,), fill, dtype=torch.uint8, device="cuda")
    m = fo.Matrices(rp.size - 1, phantom.n_cols, int(rp[-1]), *[fo._ptr(t) for t in arrays],
                    storage, 1, 0, reserve)
    h = ct.c_void_p()
    fo._check(fo.lib().fredopt_load_matrices(ct.byref(m), fo._ptr(ws), nbytes, None,
                                             ct.byref(h)))
    torch.cuda.synchronize()
    plan = fo.Plan(h, ws, rp.size - 1, phantom.n_cols, int(rp[-1]), storage)
    prob = fo.DeviceProblem(phantom.problem_arrays(), phantom.c)
    x0 = torch.from_numpy(np.ascontiguousarray(phantom.x0, np.float32)).cuda()
    return plan, prob, x0
