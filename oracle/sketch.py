"""The sparse-sign subspace embedding S (Section 2.1, eq. sparse_sign_sketch).

S = zeta^(-1/2) [s_1 ... s_n] in R^{d x n}; column j has exactly zeta nonzeros
equal to +-1 (Rademacher), placed in zeta *distinct* rows chosen uniformly at
random.  The paper draws them from PCG64DXSM and stores S (appendix); here S is
defined by a counter-based generator so that any column can be regenerated
anywhere (reading: distinct rows, uniform, signs equiprobable).

Specification (shared with the HIP library, implemented there independently):

* key = (seed & 0xffffffff, seed >> 32);
* block b of column j is Philox4x32-7 of counter (j & 0xffffffff, j >> 32, b, 0)
  (seven rounds; see ``philox``);
* row draws: word (l mod 4) of block (l div 4), l = 0..zeta-1;
* rows by Floyd's algorithm: for l = 0..zeta-1 let J = d - zeta + l and
  r = floor(word_l * (J+1) / 2^32) in [0, J]; if r is already taken the slot
  takes J, otherwise r.  This yields a uniformly random zeta-subset with a
  fixed number of draws (the multiply-shift draw has relative bias < 2^-24);
* signs: bit 0 of row draw l: 0 -> +1, 1 -> -1.  Given the row r, the draw lies
  in an interval of at least 2^32 / 65536 consecutive words, so its lowest bit
  is even or odd with probabilities within 2^-17 of 1/2 (d <= 65536).

zeta <= 32 and zeta <= d are required.
"""
import numpy as np
import scipy.sparse as sp

from .philox import philox4x32_7


def rows_and_signs(col0: int, count: int, d: int, zeta: int, seed: int):
    """(rows[count, zeta] int64, signs[count, zeta] float64 of +-1) for columns col0..col0+count-1."""
    if not (1 <= zeta <= 32 and zeta <= d):
        raise ValueError("need 1 <= zeta <= min(32, d)")
    cols = np.arange(col0, col0 + count, dtype=np.uint64)
    lo, hi = cols & np.uint64(0xFFFFFFFF), cols >> np.uint64(32)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    nblk = (zeta + 3) // 4
    words = []
    for b in range(nblk):
        out = philox4x32_7(lo, hi, np.full_like(lo, b), np.zeros_like(lo), k0, k1)
        words.extend(out)
    rows = np.empty((count, zeta), dtype=np.int64)
    for l in range(zeta):
        J = d - zeta + l
        r = ((words[l] * np.uint64(J + 1)) >> np.uint64(32)).astype(np.int64)
        taken = np.zeros(count, dtype=bool)
        for q in range(l):
            taken |= rows[:, q] == r
        rows[:, l] = np.where(taken, J, r)
    bits = np.stack([words[l] & np.uint64(1) for l in range(zeta)], axis=1)
    signs = 1.0 - 2.0 * bits.astype(np.float64)
    return rows, signs


def sketch_matrix(n: int, d: int, zeta: int, seed: int, chunk: int = 1 << 20) -> sp.csr_matrix:
    """Assemble S (d x n) as a scipy sparse matrix, column by column per the spec."""
    rr, cc, vv = [], [], []
    scale = 1.0 / np.sqrt(zeta)
    for c0 in range(0, n, chunk):
        cnt = min(chunk, n - c0)
        rows, signs = rows_and_signs(c0, cnt, d, zeta, seed)
        rr.append(rows.ravel())
        cc.append(np.repeat(np.arange(c0, c0 + cnt, dtype=np.int64), zeta))
        vv.append((signs * scale).ravel())
    return sp.csr_matrix((np.concatenate(vv), (np.concatenate(rr), np.concatenate(cc))), shape=(d, n))
