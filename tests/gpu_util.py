"""Helpers for the GPU parity tests: device copies of seeded inputs and the
tolerances the tests state."""
import numpy as np
import torch

DEV = "cuda:0"
U64 = 2.0 ** -53
U32 = 2.0 ** -24

TORCH_IDX = {"i32": torch.int32, "i64": torch.int64}


def gamma(m, u):
    mu = np.asarray(m, np.float64) * u
    return mu / (1.0 - mu)


def dev_csr(spk, A, ptr="i64", idx="i32", val=torch.float64, values=None):
    """Device CSR descriptor for host CSR A (values optionally overridden)."""
    rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, np.int64)).to(TORCH_IDX[ptr]).to(DEV)
    ci = torch.from_numpy(np.ascontiguousarray(A.col, np.int64)).to(TORCH_IDX[idx]).to(DEV)
    v = A.val if values is None else values
    va = torch.from_numpy(np.ascontiguousarray(v, np.float64)).to(val).to(DEV)
    return spk.CsrMatrix(rp, ci, va, A.n_rows, A.n_cols)


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(dtype).to(DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
