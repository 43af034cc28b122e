// Internal declarations of libfab (device code for gfx950 and the host driver).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <type_traits>

namespace fab {

constexpr int kThreads = 256;      // threads per block of the streaming kernels
constexpr int kSlots = 8;          // copies of each accumulator of the plain comparator's atomics
constexpr int kMaxParts = 2048;    // largest grid of a kernel that writes per-block partial sums
constexpr int kMaxM = 64;          // largest cycle length
constexpr int kMaxD = 4096;        // largest sketch dimension (LDS bins: 4 x 32 KB FP64 per block)
constexpr int kMaxNt = 16;         // largest number of time points per solve
constexpr int kRuleMain = 128;     // default nodes of the quadrature rule
constexpr int kRuleCosSqrt = 256;  // default nodes of the ellipse rule of cos(t sqrt z)
constexpr int kRuleSamples = 256;  // sample points of the rule's accuracy check
constexpr double kExpP = 3.0, kExpMu = 6.0, kExpL = 45.0;  // parabolic contour of the exp rule
constexpr int kXcds = 8;           // MI355X: 8 accelerator complex dies, each with its own L2
constexpr int kMaxBatch = 1024;    // largest number of right-hand sides per batched solve
constexpr int kGrowRows = 1024;    // largest growing block matrix (cycles x m) of the growing restart
constexpr int kGrowMaxSteps = 1 << 14;  // Taylor steps of exp(-t M) e_1 beyond which the restart gives up
constexpr double kDivergedEst = 1e8;  // ||y|| / ||x|| above which a member's solve is abandoned

// ----------------------------------------------------------------------------------------------
// Sparse-sign sketch specification (eq. sparse_sign_sketch): column j of S has zeta distinct
// rows chosen uniformly (Floyd's sampling algorithm) and Rademacher signs, all drawn from the
// counter-based generator Philox4x32 (Salmon et al., SC'11) with seven rounds, the fewest its
// authors report to pass their statistical test batteries (their standard form has ten):
//   key = (seed lo, seed hi); block b of column j = Philox(counter = (j lo, j hi, b, 0));
//   draw l = word (l mod 4) of block (l div 4); row J = d-zeta+l candidate r = mulhi(draw, J+1),
//   replaced by J if already taken; sign = bit 0 of draw l (1 = negative).  Given r, a draw
//   spans at least 2^32 / d consecutive words, so its low bit is nearly unbiased and independent
//   of the row; two blocks per column (zeta = 8) instead of three with a separate sign block.
// ----------------------------------------------------------------------------------------------
constexpr int kPhiloxRounds = 7;
__device__ __forceinline__ void philox4x32(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                           uint32_t k1) {
#pragma unroll
  for (int r = 0; r < kPhiloxRounds; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // each 32 x 32 -> 64-bit product as one 64-bit multiply (a single v_mad_u64_u32 gives both
    // halves; separate high and low multiplies would cost two quarter-rate instructions)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Rows and signs of column `col`; only the first `zeta` (<= ZMAX) entries are meaningful.
template <int ZMAX>
__device__ __forceinline__ void sketch_column(uint64_t col, int d, int zeta, uint32_t k0, uint32_t k1,
                                              int (&rows)[ZMAX], uint32_t& signbits) {
  uint32_t words[ZMAX];
  const uint32_t lo = (uint32_t)col, hi = (uint32_t)(col >> 32);
#pragma unroll
  for (int b = 0; b < (ZMAX + 3) / 4; ++b) {
    uint32_t c0 = lo, c1 = hi, c2 = (uint32_t)b, c3 = 0u;
    if (4 * b < zeta) philox4x32(c0, c1, c2, c3, k0, k1);
    if (4 * b + 0 < ZMAX) words[4 * b + 0] = c0;
    if (4 * b + 1 < ZMAX) words[4 * b + 1] = c1;
    if (4 * b + 2 < ZMAX) words[4 * b + 2] = c2;
    if (4 * b + 3 < ZMAX) words[4 * b + 3] = c3;
  }
  signbits = 0u;
#pragma unroll
  for (int l = 0; l < ZMAX; ++l) signbits |= (words[l] & 1u) << l;
#pragma unroll
  for (int l = 0; l < ZMAX; ++l) {
    if (l < zeta) {
      const uint32_t J = (uint32_t)(d - zeta + l);
      const int r = (int)__umulhi(words[l], J + 1u);
      bool taken = false;
#pragma unroll
      for (int q = 0; q < l; ++q) taken |= (rows[q] == r);
      rows[l] = taken ? (int)J : r;
    } else {
      rows[l] = 0;
    }
  }
}

// ----------------------------------------------------------------------------------------------
// Small complex arithmetic (FP64) for the quadrature solves.
// ----------------------------------------------------------------------------------------------
struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmk(double r, double i) { return cplx{r, i}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx cscale(cplx a, double s) { return cplx{a.re * s, a.im * s}; }
// principal square root (branch cut on the negative real axis), without cancellation
__device__ __forceinline__ cplx csqrt_p(cplx z) {
  const double r = hypot(z.re, z.im);
  if (r == 0.0) return cplx{0.0, 0.0};
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return cplx{t, z.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - z.re));
  return cplx{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}
// cos(x + iy) = cos x cosh y - i sin x sinh y
__device__ __forceinline__ cplx ccos(cplx z) { return cplx{cos(z.re) * cosh(z.im), -sin(z.re) * sinh(z.im)}; }
// Functions whose rule is conjugate-symmetric: only the Im zeta > 0 half of the nodes is kept and
// the sums take twice the real part (all but z^(-1/2), whose nodes are real).
__host__ __device__ __forceinline__ bool rule_is_half(int fun) { return fun != 1; }
__device__ __forceinline__ double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }
// a / b, scaled to avoid overflow (Smith's method)
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    const double r = b.re / b.im, den = b.re * r + b.im;
    return cplx{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}

// ----------------------------------------------------------------------------------------------
// Device-resident solver state (one per solve; FP64).
// ----------------------------------------------------------------------------------------------
struct State {
  double alpha, inv_alpha, beta, h, cpl;  // cpl = alpha r_{m+1,m} tau: restart coupling of psi
  double upd_coef[kMaxM + 1];   // window coefficients r_ij of the current step (index i - lo)
  double inv_rho, raw2;
  int meff, brk, nonfinite, step_lo;
  // per-cycle outputs read by the host
  double ynorm2[kMaxNt], xnorm2[kMaxNt];
  double est, rule_err;
  double kappa_T;       // max_i T_ii / min_i T_ii of the cycle's whitening factor
  int converged, done;  // done: converged, broken down or non-finite; every kernel skips the member
  // growing restart: alpha of cycle 1, r tau of the last cycle appended, cycles and rows so far,
  // and whether exp(-t M) e_1 needed more than kGrowMaxSteps Taylor steps
  double grow_alpha1, grow_rt;
  int grow_c, grow_p, grow_fail;
  int gram_rows;  // rows of the sketched Gram matrix G = U^T U complete in this cycle (0: none kept)
  int whiten_chol;  // this cycle's T: 1 from the Cholesky factor of G, 0 from the Householder QR
  // stopping test: ||y_t|| of the previous cycle, the contraction ratios ||y_t|| / ||y_t||_prev of
  // the previous two cycles, the estimate with which a time point passed (0 until it has), the
  // cycles run so far, and the largest relative increment ||y_t|| / ||x_t|| of this cycle
  double yprev[kMaxNt], qprev[kMaxNt], qprev2[kMaxNt], passed[kMaxNt];
  double relupd;
  int cyc;
  int passed_mask;  // bit t: time point t has passed the test
};

// Host-visible per-cycle report (copied to pinned memory each cycle).
struct Report {
  double est, rule_err, alpha, beta, kappa_T, relupd;
  int brk, meff, nonfinite, converged, done, grow_fail;
};

// Per-block partial sums in a fixed order.  A kernel whose grid is a multiple of kXcds and at most
// kMaxParts blocks writes entry e of block b's partial to parts[e * kMaxParts + part_index()]; the
// reduction kernel then adds the entries p = 0, 1, ... in one order on every run, so the result
// does not depend on which block finished first (FP64 atomics would make it depend on that).
// Blocks are dealt round-robin to the XCDs, so the index is XCD-major: the 16 partials that share
// a 128-byte line come from blocks of one XCD and merge in its L2.
__device__ __forceinline__ size_t part_index() {
  return (size_t)(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
}

// Batched solves: member r of a batch owns a copy of the single-solve workspace at byte offset
// r * bs; kernels launched with gridDim.y = members shift their workspace pointers with bat().
// (Byte arithmetic on a char pointer, not an integer, so the compiler still sees a pointer derived
// from the kernel argument and keeps global-memory instructions.)
template <typename P>
__device__ __forceinline__ P* bat(P* p, size_t bs, int r) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(p) + (size_t)r * bs);
}
template <typename P>
__device__ __forceinline__ P* bat(P* p, size_t bs) {
  return bat(p, bs, (int)blockIdx.y);
}

// Column stride of the basis W, in elements of es bytes: n rounded up to whole 4 KiB pages, and an
// odd number of pages.  Columns a power of two apart (2^21 doubles are 16 MiB) start on the same
// HBM channels, and the kernels that stream several columns in step (the window update, the pass)
// then lose 5-9% of their bandwidth on MI355X.
__host__ __device__ __forceinline__ size_t wcol(int64_t n, int es) {
  const int64_t per = 4096 / es;
  int64_t pages = (n + per - 1) / per;
  if ((pages & 1) == 0) ++pages;
  return (size_t)(pages * per);
}

// Arguments of the cycle-end kernel.
struct SmallArgs {
  int d, m, nt, plain, fun, nq;
  const double* U;
  double* Uq;       // d x (m+1) scratch for the Householder QR
  const double* R;  // (m+1) x m
  double* Tout;     // (m+1) x (m+1)
  double* Xout;     // m x m: Rt = R_m + r_{m+1,m} T_m^{-1} t e_m^T (similar to the whitened X)
  const cplx* rz;
  const cplx* rw;
  cplx* psi;
  double* gbuf;     // (nt nq) x m: each rule node's term of the restart coefficients (k_combine adds them)
  double* C;        // (m+1) x (nt+1) pass coefficients (main rule), restart column last
  const double* G;  // (m+1) x (m+1) sketched Gram matrix, row-major lower triangle (st->gram_rows rows)
  State* st;
  size_t bs;        // batch stride in bytes (member blockIdx.y works at byte offset blockIdx.y * bs)
};

__device__ __forceinline__ SmallArgs member_args(const SmallArgs& a0) {
  SmallArgs a = a0;
  const size_t bs = a0.bs;
  a.U = bat(a0.U, bs);
  a.Uq = bat(a0.Uq, bs);
  a.R = bat(a0.R, bs);
  a.Tout = bat(a0.Tout, bs);
  a.Xout = bat(a0.Xout, bs);
  a.rz = bat(a0.rz, bs);
  a.rw = bat(a0.rw, bs);
  a.psi = bat(a0.psi, bs);
  a.gbuf = bat(a0.gbuf, bs);
  a.C = bat(a0.C, bs);
  a.G = bat(a0.G, bs);
  a.st = bat(a0.st, bs);
  return a;
}

// Sketch of the restart vector formed by the pass for the next cycle's start (on == 0: the pass
// does not sketch, and the cycle starts with a sketch-only pass instead).  The pass writes its
// partials of S v_hat to entries [0, d) of the partial buffer and those of the norms after them.
struct PassSketch {
  int on;
  int d, zeta;    // zeta <= 8
  uint32_t k0, k1;
  double scale;   // 1/sqrt(zeta) rounded to the value type, as the sketch-only pass applies it
};

// Workspace carving, shared by the driver and workspace_size().
// Workspace of the growing restart (one member): blocks, couplings and sizes per cycle.
struct GrowBuffers {
  double* M;
  double* K;
  int* sz;
  const double* tvals;
};

struct Layout {
  size_t W, U, R, slots_step, slots_start, uraw, red, state, T, Ut, X, C, rule_z, rule_w, psi, gbuf, grow, G,
      parts, total;
  int nsys, nq;
};

}  // namespace fab
