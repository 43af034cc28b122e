"""Finite-difference PDE operators in CSR form (inputs only, no solver arithmetic).

Conventions (one reading, used everywhere in this repository):

* unit square / cube, homogeneous Dirichlet boundary, interior nodes only,
  mesh width ``h = 1/(N+1)``, lexicographic ordering with x fastest:
  ``row = ix + N*iy (+ N*N*iz)``;
* every stencil is scaled by ``h**-2`` (convection by ``h**-1``);
* columns inside a row are sorted ascending; ``rowptr``/``colind`` are int32.

The operators are Kronecker sums of one-dimensional tridiagonal factors
(``A = T_x (+) T_y (+) T_z`` plus an optional shift), which is what lets the
oracle compute f(A)b in closed form.  The factor coefficients are given here
as plain numbers (sub-, main-, super-diagonal per axis) so that the CSR can be
assembled without any dense linear algebra.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class CSR:
    """A square sparse matrix in CSR form with int32 indices."""
    n: int
    rowptr: np.ndarray          # int32, n+1
    colind: np.ndarray          # int32, nnz
    vals: np.ndarray            # float64 (or float32), nnz
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def astype(self, dtype) -> "CSR":
        return CSR(self.n, self.rowptr, self.colind, self.vals.astype(dtype), dict(self.meta))

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))


def stencil_csr(N: int, dim: int, axis_coeffs, shift: float = 0.0, dtype=np.float64) -> CSR:
    """Assemble ``sum_d I (x) .. (x) T_d (x) .. (x) I + shift*I`` on an N^dim grid.

    ``axis_coeffs[d] = (lo, diag, hi)`` are the entries of the 1-D factor of
    axis ``d`` (d=0 is x, the fastest index): ``T_d[i,i-1] = lo``,
    ``T_d[i,i] = diag``, ``T_d[i,i+1] = hi``.
    """
    assert dim in (1, 2, 3) and len(axis_coeffs) == dim
    n = N ** dim
    idx = np.arange(n, dtype=np.int64)
    coords = [(idx // (N ** d)) % N for d in range(dim)]
    center = float(sum(c[1] for c in axis_coeffs)) + float(shift)
    # offsets in ascending column order: -N^(dim-1) ... -1, 0, +1 ... +N^(dim-1)
    entries = []
    for d in reversed(range(dim)):
        entries.append((-(N ** d), d, 0))
    entries.append((0, None, 1))
    for d in range(dim):
        entries.append((N ** d, d, 2))
    masks = []
    for off, d, which in entries:
        if d is None:
            masks.append(np.ones(n, dtype=bool))
        elif off < 0:
            masks.append(coords[d] > 0)
        else:
            masks.append(coords[d] < N - 1)
    counts = np.zeros(n, dtype=np.int64)
    for mk in masks:
        counts += mk
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    if nnz >= 2 ** 31:
        raise ValueError("nnz exceeds int32 range")
    colind = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=dtype)
    cursor = rowptr[:-1].copy()
    for (off, d, which), mk in zip(entries, masks):
        rows = idx[mk]
        pos = cursor[mk]
        colind[pos] = (rows + off).astype(np.int32)
        vals[pos] = center if d is None else axis_coeffs[d][0 if off < 0 else 2]
        cursor[mk] += 1
    return CSR(n, rowptr.astype(np.int32), colind, vals,
               {"N": N, "dim": dim, "axis_coeffs": [tuple(map(float, c)) for c in axis_coeffs],
                "shift": float(shift)})


def _lap_coeffs(N: int, scale: float = 1.0):
    h = 1.0 / (N + 1)
    return (-scale / h ** 2, 2.0 * scale / h ** 2, -scale / h ** 2)


def laplacian_2d(N: int, dtype=np.float64) -> CSR:
    """-Delta_h with the 5-point stencil on an N x N interior grid (n = N^2)."""
    A = stencil_csr(N, 2, [_lap_coeffs(N)] * 2, dtype=dtype)
    A.meta["name"] = f"laplacian_2d_N{N}"
    return A


def anisotropic_2d(N: int, cy: float = 0.01, dtype=np.float64) -> CSR:
    """-d_xx - cy d_yy with the 5-point stencil (n = N^2)."""
    A = stencil_csr(N, 2, [_lap_coeffs(N), _lap_coeffs(N, cy)], dtype=dtype)
    A.meta["name"] = f"anisotropic_2d_N{N}_cy{cy}"
    return A


def convdiff_3d(N: int, peclet: float, dtype=np.float64) -> CSR:
    """-Delta_h + Pe (d_x + d_y + d_z)_h, central differences, wind (1,1,1).

    Row i of each 1-D factor: ``(-1/h^2 - Pe/(2h)) u[i-1] + 2/h^2 u[i]
    + (-1/h^2 + Pe/(2h)) u[i+1]``.  Non-symmetric for Pe != 0.
    """
    h = 1.0 / (N + 1)
    c = (-1.0 / h ** 2 - peclet / (2 * h), 2.0 / h ** 2, -1.0 / h ** 2 + peclet / (2 * h))
    A = stencil_csr(N, 3, [c] * 3, dtype=dtype)
    A.meta["name"] = f"convdiff_3d_N{N}_Pe{peclet:g}"
    return A


def shifted_laplacian_3d(N: int, shift: float = 1.0, dtype=np.float64) -> CSR:
    """-Delta_h + shift*I with the 7-point stencil (SPD), n = N^3."""
    A = stencil_csr(N, 3, [_lap_coeffs(N)] * 3, shift=shift, dtype=dtype)
    A.meta["name"] = f"shifted_laplacian_3d_N{N}_s{shift:g}"
    return A


def ragged_laplacian_sizes(count: int = 32, lo: int = 64, hi: int = 512):
    """Grid sizes log-spaced from lo to hi: N_i = round(lo * (hi/lo)^(i/(count-1)))."""
    return [int(round(lo * (hi / lo) ** (i / (count - 1)))) for i in range(count)]
