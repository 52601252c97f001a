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
