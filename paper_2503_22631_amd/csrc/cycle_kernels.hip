// Cycle-level kernels: quadrature nodes, cycle start, the cycle-end small FP64 work (whitening
// QR, projected matrix, quadrature restart), the fused tall-skinny pass and the convergence test.
//
// Whitening (appendix, eq. A.1): S W_{m+1} = Q T_{m+1}, T = [[T_m, t], [0, tau]], diag(T) > 0;
//   X = T_m R_m T_m^{-1} + (r_{m+1,m}/T_m[m,m]) t e_m^T,  h = r_{m+1,m} tau / T_m[m,m],
//   so A V = V X + h v_hat e_m^T with V = W_m T_m^{-1}, v_hat = (w_{m+1} - V t)/tau (an Arnoldi-like
//   decomposition, eq. rand_arnoldi), and the start vector is beta V e_1 with beta = alpha T[1,1].
// Restart (Algorithm 2 with f of the growing matrix replaced by a quadrature rule
//   r(z) = sum_l w_l/(zeta_l - z)): block c of r(M_c) e_1 is
//   g_c = beta_c sum_l w_l psi_l (zeta_l I - X)^{-1} e_1,   psi_l <- psi_l beta_c h_c [(zeta_l - X)^{-1} e_1]_m,
//   by block forward substitution of the block lower-bidiagonal M_c (eq. restart_combined).
// The pass then adds x_t += W_m (T_m^{-1} g_t) and forms v_hat in one read of the basis.
// The growing restart (k_grow_append, k_grow_expmv) evaluates exp on M_c itself instead, as
// Algorithm 2 states it.
#include "fab_internal.h"

namespace fab {

__device__ __forceinline__ double wave_sum_c(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
// Value of v in lane i (i the same in every lane), through the scalar unit.
__device__ __forceinline__ double bcast_lane(double v, int i) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, i);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), i);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Fill a double buffer with zeros (used instead of memset so the same code can sit in a graph).
__global__ void k_zero(double* p, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

// count doubles at p + blockIdx.y * step_bytes, for every y (batch members, or columns of x).
__global__ void k_zero_strided(double* p, size_t count, size_t step_bytes) {
  p = bat(p, step_bytes);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

// ------------------------------------------------------------------------------- quadrature rules
// fun 0, exp(-t z): parabolic Hankel contour s(u) = P - mu u^2 + 2 i mu u, u in [-U, U],
//   U = sqrt((P+L)/mu), N midpoint nodes; zeta = -s/t, w = -h s'(u) e^s / (2 pi i t).  Only the
//   nodes with u < 0 (Im zeta > 0) are kept: for real X the other half are conjugates, and the
//   accumulation takes twice the real part.  (N, P, mu, L) = (N, 3, 6, 45).
// fun 2, phi_1(-t z) (eq. conv_diff_sol3): the same contour and nodes, each weight divided by its
//   s = -t zeta.  The integral of e^s / (s (s - s0)) over a contour around 0 and s0 is phi_1(s0)
//   (residues at 0 and s0), and e^s / s decays on the contour's tails like e^s.
// fun 1, z^(-1/2) = (2/pi) int_0^inf (z + s^2)^{-1} ds with s = c tan(theta), N midpoint nodes on
//   (0, pi/2): zeta = -c^2 tan^2(theta), w = -(c/N) sec^2(theta), c = (lo hi)^(1/4).
// fun 3, cos(t sqrt z) (eq. drum_sol): Cauchy integral on the ellipse zeta(theta) = c + h (rho e^{i
//   theta} + e^{-i theta} / rho) / 2 around [lo, hi] (c, h its centre and half-width), trapezoidal
//   nodes theta = 2 pi (k + 1/2) / N, w = f(zeta) zeta'(theta) / (i N), rho from cos_rule_rho.
//   cos(t sqrt z) is entire, so no branch of the square root matters.  The Im zeta > 0 half
//   (theta < pi) is kept, as for exp.
// Layout: nq nodes per time point (nq = N/2 for the conjugate-half rules, N for z^(-1/2)).
// The ellipse of the cos(t sqrt z) rule.  For a point z with ellipse coordinate |w(z)| < rho
// (z = c + h (w + 1/w) / 2) the truncation error falls like (|w(z)| / rho)^N, and the points that
// matter are the eigenvalues of the cycles' projected matrices: sketched Ritz values, which can fall
// slightly outside [lo, hi] because the sketched projection is oblique.  The rounding of the sum
// grows with max |f| on the ellipse, i.e. with t max |Im sqrt zeta|.  rho_min = exp(37 / N) is the
// smallest ellipse with rho^-N below FP64 rounding; the rule takes the largest candidate
// rho_min (cap / rho_min)^(j / kCosRhoSteps), j = kCosRhoSteps .. 0, cap = max(2, rho_min), whose
// growth t max_k |Im sqrt zeta_k| over its Im zeta > 0 nodes stays within max(ln 100, the growth
// at rho_min).  A wavefront's lanes share the nodes; every lane returns the same rho.
constexpr int kCosRhoSteps = 16;
__device__ double cos_rule_rho(double t, int N, double lo, double hi, int lane) {
  const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
  const double rho_min = exp(37.0 / N), cap = fmax(2.0, rho_min);
  auto growth = [&](double rho) {
    const double ap = 0.5 * (rho + 1.0 / rho), am = 0.5 * (rho - 1.0 / rho);
    double g = 0.0;
    for (int k = lane; k < N / 2; k += 64) {
      const double th = 2.0 * M_PI * (k + 0.5) / N;
      g = fmax(g, fabs(csqrt_p(cmk(c + h * ap * cos(th), h * am * sin(th))).im));
    }
    return t * wave_max(g);
  };
  const double bound = fmax(log(100.0), growth(rho_min));
  for (int j = kCosRhoSteps; j > 0; --j) {
    const double rho = rho_min * pow(cap / rho_min, (double)j / kCosRhoSteps);
    if (growth(rho) <= bound) return rho;
  }
  return rho_min;
}

__global__ void k_rule(int fun, int nt, const double* __restrict__ tvals, int n_main, double lo, double hi,
                       cplx* __restrict__ rz, cplx* __restrict__ rw, cplx* __restrict__ psi, size_t bs) {
  __shared__ double s_rho[kMaxNt];
  rz = bat(rz, bs);  // every batch member holds its own copy (psi is per member)
  rw = bat(rw, bs);
  psi = bat(psi, bs);
  if (fun == 3) {  // the ellipse of each time point, by the first wavefront of every block
    if (threadIdx.x < 64)
      for (int it = 0; it < nt; ++it) {
        const double rho = cos_rule_rho(tvals[it], n_main, lo, hi, (int)threadIdx.x);
        if (threadIdx.x == 0) s_rho[it] = rho;
      }
    __syncthreads();
  }
  const int nq = rule_is_half(fun) ? n_main / 2 : n_main;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nt * nq; s += gridDim.x * blockDim.x) {
    const int it = s / nq, idx = s % nq;
    cplx z, w;
    if (fun == 0 || fun == 2) {
      const double t = tvals[it];
      const int N = n_main;
      const double P = kExpP, mu = kExpMu, L = kExpL;
      const double U = sqrt((P + L) / mu), h = 2.0 * U / N;
      const double u = -U + (idx + 0.5) * h;
      const cplx sv = cmk(P - mu * u * u, 2.0 * mu * u);
      const cplx ds = cmk(-2.0 * mu * u, 2.0 * mu);
      const double er = exp(sv.re);
      const cplx es = cmk(er * cos(sv.im), er * sin(sv.im));
      z = cscale(sv, -1.0 / t);
      // w = -h ds e^s / (2 pi i t) = (h / (2 pi t)) * i * ds * e^s
      const cplx q = cmul(ds, es);
      const double f = h / (2.0 * M_PI * t);
      w = cmk(-q.im * f, q.re * f);
      if (fun == 2) w = cdiv(w, sv);  // phi_1: weight over s (s != 0: Re s = P at u = 0)
    } else if (fun == 3) {
      const double t = tvals[it];
      const int N = n_main;
      const double rho = s_rho[it], c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
      const double th = 2.0 * M_PI * (idx + 0.5) / N;
      const double ct = cos(th), st = sin(th);
      const double ap = 0.5 * (rho + 1.0 / rho), am = 0.5 * (rho - 1.0 / rho);
      z = cmk(c + h * ap * ct, h * am * st);
      const cplx dz = cmk(-h * ap * st, h * am * ct);  // d zeta / d theta
      const cplx sq = csqrt_p(z);
      const cplx fz = ccos(cmk(t * sq.re, t * sq.im));
      const cplx q = cmul(fz, dz);
      w = cmk(q.im / N, -q.re / N);  // q / (i N)
    } else {
      const int N = n_main;
      const double c = sqrt(sqrt(lo * hi));
      const double th = (idx + 0.5) * (0.5 * M_PI) / N;
      const double tn = tan(th), cs = cos(th);
      z = cmk(-(c * tn) * (c * tn), 0.0);
      w = cmk(-(c / N) / (cs * cs), 0.0);
    }
    rz[s] = z;
    rw[s] = w;
    psi[s] = cmk(1.0, 0.0);
  }
}

// Accuracy of the rule as a function, once per solve: the restarted iteration with a fixed rule r
// converges to r(A) b, so |r - f| over the spectral region bounds what the rule adds to the error.
// Samples (kRuleSamples per time point): exp(-t z) and phi_1(-t z) at t z = 0 and t z geometric in
// [1e-4, 1e4], absolute error (0 < f <= 1 there); z^(-1/2) at z geometric in [lo, hi], relative
// error; cos(t sqrt z) at sqrt z uniform in [sqrt lo, sqrt hi], absolute error (|f| <= 1).  The
// largest error over samples and time points goes to st->rule_err.  One block of kRuleSamples threads.
__global__ __launch_bounds__(kRuleSamples) void k_rule_check(int fun, int nt, const double* __restrict__ tvals,
                                                             int nq, double lo, double hi,
                                                             const cplx* __restrict__ rz,
                                                             const cplx* __restrict__ rw, State* __restrict__ st,
                                                             int nb, size_t bs) {
  __shared__ double red[kRuleSamples / 64];
  const int j = threadIdx.x;
  double err = 0.0;
  for (int it = 0; it < nt; ++it) {
    const cplx* zz = rz + (size_t)it * nq;
    const cplx* ww = rw + (size_t)it * nq;
    double z, f;
    if (fun == 0 || fun == 2) {
      const double t = tvals[it];
      const double tz = (j == 0) ? 0.0 : 1e-4 * pow(1e8, (double)(j - 1) / (kRuleSamples - 2));
      z = tz / t;
      f = (fun == 0) ? exp(-tz) : (tz > 0.0 ? -expm1(-tz) / tz : 1.0);
    } else if (fun == 3) {
      const double t = tvals[it];
      const double sq = sqrt(lo) + (sqrt(hi) - sqrt(lo)) * (double)j / (kRuleSamples - 1);
      z = sq * sq;
      f = cos(t * sq);
    } else {
      z = lo * pow(hi / lo, (double)j / (kRuleSamples - 1));
      f = 1.0 / sqrt(z);
    }
    cplx r = cmk(0.0, 0.0);
    // four independent divisions per trip, so their dependent chains interleave
#pragma unroll 4
    for (int l = 0; l < nq; ++l) r = cadd(r, cdiv(ww[l], csub(zz[l], cmk(z, 0.0))));
    const double rv = rule_is_half(fun) ? 2.0 * r.re : r.re;  // conjugate-half rules: twice the real part
    err = fmax(err, (fun == 1) ? fabs(rv / f - 1.0) : fabs(rv - f));
  }
  for (int off = 32; off > 0; off >>= 1) err = fmax(err, __shfl_xor(err, off, 64));
  if ((j & 63) == 0) red[j >> 6] = err;
  __syncthreads();
  if (j == 0) {
    double e = 0.0;
    for (int q = 0; q < kRuleSamples / 64; ++q) e = fmax(e, red[q]);
    for (int r = 0; r < nb; ++r) bat(st, bs, r)->rule_err = e;
  }
}

template <typename T>
__global__ void k_copy_in(int n, const T* __restrict__ b, int64_t ldb, T* __restrict__ w0, size_t bs) {
  b += (int64_t)blockIdx.y * ldb;
  w0 = bat(w0, bs);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += stride) w0[i] = b[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sqnorm(int n, const T* __restrict__ v, double* __restrict__ slots) {
  __shared__ double part[kThreads / 64];
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < (size_t)n; i += stride) {
    const double x = (double)v[i];
    acc += x * x;
  }
  acc = wave_sum_c(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += part[q];
    unsafeAtomicAdd(slots + (blockIdx.x % kSlots), s);
  }
}

// Cycle start (the normalisation that opens Algorithm 1): alpha = ||S v|| and u_1 = S v / alpha
// (sketched; sv = S v, the fixed-order sum of the partials), or alpha = ||v|| (plain: kSlots copies
// of ||v||^2 in slots_start).  Resets the per-cycle flags; for the plain method also zeroes its
// accumulators.
__global__ __launch_bounds__(kThreads) void k_start(int d, int m, int plain, const double* __restrict__ sv,
                                                    double* __restrict__ slots_start,
                                                    double* __restrict__ slots_step, size_t step_len,
                                                    double* __restrict__ U, double* __restrict__ R,
                                                    State* __restrict__ st, size_t bs) {
  __shared__ double part[kThreads / 64];
  __shared__ double s_alpha;
  st = bat(st, bs);
  if (st->done) return;
  slots_start = bat(slots_start, bs);
  slots_step = bat(slots_step, bs);
  sv = bat(sv, bs);
  U = bat(U, bs);
  R = bat(R, bs);
  double acc = 0.0;
  if (!plain) {
    for (int i = threadIdx.x; i < d; i += kThreads) {
      const double s = sv[i];
      U[i] = s;
      acc += s * s;
    }
  } else if (threadIdx.x < kSlots) {
    acc = slots_start[threadIdx.x];
  }
  acc = wave_sum_c(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += part[q];
    const double alpha = sqrt(s);
    s_alpha = alpha;
    st->alpha = alpha;
    st->inv_alpha = (alpha > 0.0) ? 1.0 / alpha : 0.0;
    st->meff = m;
    st->brk = 0;
    st->nonfinite = 0;
    st->gram_rows = 0;
    if (!isfinite(alpha)) {
      st->nonfinite = 1;
      st->brk = 1;
      st->meff = 0;
    } else if (!(alpha > 0.0)) {  // v = 0: nothing to add, the solve is finished exactly
      st->brk = 1;
      st->meff = 0;
    }
  }
  __syncthreads();
  const double inv = (s_alpha > 0.0) ? 1.0 / s_alpha : 0.0;
  if (!plain) {
    for (int i = threadIdx.x; i < d; i += kThreads) U[i] *= inv;
  } else {
    for (int i = threadIdx.x; i < kSlots; i += kThreads) slots_start[i] = 0.0;
    for (size_t i = threadIdx.x; i < 2 * step_len; i += kThreads) slots_step[i] = 0.0;
  }
  for (int i = threadIdx.x; i < (m + 1) * m; i += kThreads) R[i] = 0.0;
}

// ------------------------------------------------------------------------- cycle-end small FP64


// ---------------------------------------------------------------------------------------------
// Cycle-end small FP64 work.
//
// With U_{m+1} = Q T_{m+1}, the whitened projected matrix X = T_m R_m T_m^{-1} + (r/T_mm) t e_m^T
// is similar to Rt = T_m^{-1} X T_m = R_m + r s e_m^T, s = T_m^{-1} t (r = r_{m+1,m}; the last row
// of T_m is T_mm e_m^T).  Rt is still upper Hessenberg, so the restart works on Rt and X is never
// formed: (zeta - X)^{-1} e_1 = T_m (zeta - Rt)^{-1} e_1 / T_11, and with beta = alpha T_11
//   c_t = T_m^{-1} g_t = alpha sum_l w_l psi_l (zeta_l - Rt)^{-1} e_1   (pass coefficients on W_m)
//   psi_l <- psi_l beta h [(zeta_l - X)^{-1} e_1]_m = psi_l alpha r tau [(zeta_l - Rt)^{-1} e_1]_m
//   v_hat = (w_{m+1} - W_m s) / tau.
// ---------------------------------------------------------------------------------------------
constexpr int kWhitenThreads = 576;  // 9 waves x 8 columns x 8 lanes: up to kMaxM + 1 columns

__device__ __forceinline__ double sum8(double v) {  // over the 8 lanes of a column group
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  return v;
}

// Common tail of the whitening kernels (T in LDS, row-major, positive diagonal; all threads arrive
// after a barrier): T to global, s = T_m^{-1} t, Rt, the restart column of the pass coefficients,
// and the scalars of the restart recursion.
__device__ void whiten_tail(const SmallArgs& a, const double* Ts, int ldT, int mm, int brk, double* s_lds) {
  State* st = a.st;  // a: this member's arguments (already offset)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = a.m, nt = a.nt, nthr = blockDim.x;
  const int cols = brk ? mm : mm + 1;
  for (int e = tid; e < (m + 1) * (m + 1); e += nthr) {
    const int i = e % (m + 1), l = e / (m + 1);  // column-major output
    a.Tout[e] = (i < cols && l < cols && l >= i) ? Ts[i * ldT + l] : 0.0;
  }
  for (int e = tid; e < nt * m; e += nthr) a.gbuf[e] = 0.0;  // rule sums of k_quad
  if (wv == 0) {  // s = T_m^{-1} t, column-oriented back substitution; lane i holds s_i
    // reciprocal diagonal in lane i; the column entries T[lane, i] are read eight columns at a time
    // ahead of the chain, whose step is then a multiply, a lane broadcast and an FMA
    const double rd = (lane < mm) ? 1.0 / Ts[lane * ldT + lane] : 0.0;
    double rhs = (!brk && lane < mm) ? Ts[lane * ldT + mm] : 0.0;
    double sl = 0.0;
    for (int i0 = mm - 1; i0 >= 0; i0 -= 8) {
      double tc[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = i0 - r;
        tc[r] = (i >= 0 && lane < i) ? Ts[lane * ldT + i] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = i0 - r;
        if (i >= 0) {
          const double si = bcast_lane(rhs * rd, i);
          if (lane == i) sl = si;
          rhs -= tc[r] * si;
        }
      }
    }
    if (lane < mm) s_lds[lane] = sl;
    // spread of T's diagonal (positive): max_i T_ii / min_i T_ii bounds cond_2(T) below
    double dmin = INFINITY, dmax = 0.0;
    for (int i = lane; i < cols; i += 64) {
      dmin = fmin(dmin, Ts[i * ldT + i]);
      dmax = fmax(dmax, Ts[i * ldT + i]);
    }
    dmin = wave_min(dmin);
    dmax = wave_max(dmax);
    if (lane == 0) st->kappa_T = dmax / dmin;
  }
  __syncthreads();
  const double r = brk ? 0.0 : a.R[(size_t)(mm - 1) * (m + 1) + mm];
  const double tau = brk ? 1.0 : Ts[mm * ldT + mm];
  for (int e0 = 0; e0 < m * m; e0 += 8 * nthr) {  // Rt, column-major with leading dimension m
    double v[8];  // eight loads of R in flight per thread
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr + tid, i = e % m, c = e / m;
      v[u] = (e < m * m && i < mm && c < mm) ? a.R[(size_t)c * (m + 1) + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr + tid, i = e % m, c = e / m;
      if (e < m * m) a.Xout[e] = v[u] + ((i < mm && c == mm - 1) ? r * s_lds[i] : 0.0);
    }
  }
  double* rcol = a.C + (size_t)nt * (m + 1);
  for (int e = tid; e <= m; e += nthr)
    rcol[e] = brk ? 0.0 : (e < mm ? -s_lds[e] / tau : (e == mm ? 1.0 / tau : 0.0));
  if (tid == 0) {
    const double alpha = st->alpha;
    st->beta = alpha * Ts[0];
    st->h = brk ? 0.0 : r * tau / Ts[(mm - 1) * ldT + (mm - 1)];
    st->cpl = brk ? 0.0 : alpha * r * tau;
  }
}

// T from the sketched Gram matrix G = U^T U = T^T T (kept row by row by the steps): LDL^T in LDS
// by columns, one barrier per column (wave w updates rows c+1+w, c+10+w, .., lane l column c+1+l),
// then T_kk = sqrt(D_k) and T_ki = L_ik sqrt(D_k).  Cholesky squares the condition number: its T
// is off by about cond_2(U)^2 eps relative, against cond_2(U) eps for the Householder QR, and the
// restarted iteration can amplify that difference (on a 256^3 z^(-1/2) solve with k = 2, a cycle
// with cond_2(U) = 3e4 left T off by 1e-9 and moved the solve from 33 to 33-91 cycles).  So the
// factor is kept only when kappa_F(T) = ||T||_F ||T^{-1}||_F, an upper bound on cond_2(U), is at
// most kCholMaxCond; T^{-1} comes from a bottom-up row solve in one wavefront (lane = column).
// Otherwise, and for a pivot below kCholMinPivot of its column's squared norm or more than 64
// columns, it returns false and the caller runs the Householder QR.  Every thread returns the same
// result.  (Measured on the 128^3 workload: 66 us per cycle end, 38 of them the LDL^T, against
// 114 us for the Householder QR.  Keeping the trailing entries in registers and publishing each
// column made the LDL^T slower, 44 us.)
constexpr double kCholMinPivot = 1e-6;
constexpr double kCholMaxCond = 1000.0;  // accepted factors stay within about 3e-13 of the Householder T

__device__ bool whiten_gram(const SmallArgs& a, int cols, double* Ts, int ldT, double* gd) {
  __shared__ double Xs[64 * 64];  // T^{-1}, row-major
  __shared__ double s_inv2;       // ||T^{-1}||_F^2
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nthr = kWhitenThreads, nwv = kWhitenThreads / 64;
  if (cols > 64) return false;  // uniform: no barrier passed yet
  const int ldg = a.m + 1;
  constexpr int kPer = ((kMaxM + 1) * (kMaxM + 1) + kWhitenThreads - 1) / kWhitenThreads;
  double gv[kPer];  // all loads in flight together: one memory latency, not one per entry
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * nthr, i = e / cols, k = e % cols;
    gv[u] = (e < cols * cols && k <= i) ? a.G[(size_t)i * ldg + k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = tid + u * nthr, i = e / cols, k = e % cols;
    if (e < cols * cols && k <= i) {
      Ts[i * ldT + k] = gv[u];
      if (k == i) gd[i] = gv[u];
    }
  }
  __syncthreads();
  for (int c = 0; c < cols; ++c) {
    const double piv = Ts[c * ldT + c];
    if (!(piv >= kCholMinPivot * gd[c]) || !(piv < INFINITY)) {  // the same outcome in every thread
      __syncthreads();  // every thread has read piv and gd[c] before the caller reuses Ts and gd
      return false;
    }
    const double inv = 1.0 / piv;
    const int k = c + 1 + lane;  // k <= c + 64 covers every column up to kMaxM
    for (int i = c + 1 + wv; i < cols; i += nwv)
      if (k <= i) Ts[i * ldT + k] -= Ts[i * ldT + c] * (Ts[k * ldT + c] * inv);
    __syncthreads();
  }
  for (int c = tid; c < cols; c += nthr) gd[c] = sqrt(Ts[c * ldT + c]);
  __syncthreads();
  for (int e = tid; e < cols * cols; e += nthr) {
    const int i = e / cols, k = e % cols;
    if (k < i) Ts[k * ldT + i] = Ts[i * ldT + k] / gd[k];  // upper triangle from the strict lower
    else if (k == i) Ts[i * ldT + i] = gd[i];
  }
  __syncthreads();
  // kappa_F(T): ||T^{-1}||_F from X = T^{-1} (upper), row i from the rows below it, X[l][c] = 0 for
  // l > c; ||T||_F from the upper triangle.  (Measured on the 128^3 workload, this kernel takes
  // 66 us; reading eight (T, X) pairs per round trip made it 122 us, and splitting each row's sum
  // over the nine waves, with a barrier per row, 78 us.)
  if (wv == 0) {
    double ss = 0.0;
    for (int i = cols - 1; i >= 0; --i) {
      double acc = (lane == i) ? 1.0 : 0.0;
      for (int l = i + 1; l < cols; ++l) acc -= Ts[i * ldT + l] * Xs[l * 64 + lane];
      const double xi = (lane >= i && lane < cols) ? acc / Ts[i * ldT + i] : 0.0;
      Xs[i * 64 + lane] = xi;
      ss += xi * xi;
    }
    ss = wave_sum_c(ss);
    if (lane == 0) s_inv2 = ss;
  }
  double ts = 0.0;
  for (int e = tid; e < cols * cols; e += nthr) {
    const int i = e / cols, l = e % cols;
    if (l >= i) ts += Ts[i * ldT + l] * Ts[i * ldT + l];
  }
  ts = wave_sum_c(ts);
  __syncthreads();  // s_inv2 written; Xs no longer read
  if (lane == 0) Xs[wv] = ts;
  __syncthreads();
  double t2 = 0.0;
  for (int q = 0; q < nwv; ++q) t2 += Xs[q];
  const bool ok = (t2 * s_inv2 <= kCholMaxCond * kCholMaxCond);  // the same values in every thread
  __syncthreads();  // every thread has read Xs and s_inv2
  return ok;
}

// Whitening QR with the sketched basis in registers (d <= 8 KR).  Column q of U is owned by the
// eight lanes 8*(q%8) .. 8*(q%8)+7 of wave q/8; lane `part` keeps rows i = part + 8k.  The
// reflector of column c is formed from the tail norm its owners accumulated in the previous step,
// the column is published in LDS (double-buffered), and every owner updates its own column in
// registers: one barrier per column.
template <int KR>
__global__ __launch_bounds__(kWhitenThreads) void k_whiten(SmallArgs a0) {
  __shared__ double Ts[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double vcol[2][8 * KR];
  __shared__ double rfs[2][2];
  __shared__ double diagR[kMaxM + 1];
  __shared__ double tail2[kMaxM + 2];
  __shared__ double s_lds[kMaxM];
  const SmallArgs a = member_args(a0);
  State* st = a.st;
  if (st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d;
  const int mm = st->meff;
  const int brk = st->brk;
  if (st->nonfinite || mm == 0) return;
  const int cols = brk ? mm : mm + 1;
  const int ldT = kMaxM + 1;
  if constexpr (KR <= 32) {  // the steps keep G only for d <= 256
    if (!a.plain && st->gram_rows >= cols && whiten_gram(a, cols, Ts, ldT, diagR)) {
      whiten_tail(a, Ts, ldT, mm, brk, s_lds);
      if (tid == 0) st->whiten_chol = 1;
      return;
    }
  }
  for (int e = tid; e < cols * cols; e += kWhitenThreads) Ts[(e / cols) * ldT + (e % cols)] = 0.0;
  __syncthreads();  // the zeros land before any entry of T is written below
  if (!a.plain) {
    const int q = wv * 8 + (lane >> 3), part = lane & 7;
    double col[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int i = part + 8 * k;
      col[k] = (q < cols && i < d) ? a.U[(size_t)q * d + i] : 0.0;
    }
    if (q == 0) {
      double s2 = 0.0;
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        vcol[0][part + 8 * k] = col[k];
        s2 += (part + 8 * k >= 1) ? col[k] * col[k] : 0.0;
      }
      s2 = sum8(s2);
      if (part == 0) tail2[0] = s2;
    }
    for (int c = 0; c < cols; ++c) {
      const int b = c & 1;
      if (q == c && part == 0) {  // reflector of column c
        const double s2 = tail2[c];
        const double alp = vcol[b][c];
        const double nrm = sqrt(alp * alp + s2);
        double tau = 0.0, beta_h = alp, scal = 0.0;
        if (s2 > 0.0 || alp < 0.0) {  // reflect unless already a nonnegative multiple of e_c
          beta_h = (alp >= 0.0) ? -nrm : nrm;
          tau = (beta_h - alp) / beta_h;
          scal = 1.0 / (alp - beta_h);
        }
        rfs[b][0] = tau;
        rfs[b][1] = scal;
        diagR[c] = beta_h;
      }
      __syncthreads();
      const double tau = rfs[b][0], scal = rfs[b][1];
      if (q > c && q < cols) {
        // H = I - tau v v^T with v = [1; U[c+1:, c] * scal].  Branch-free over the register rows:
        // every index stays inside vcol, out-of-range rows are masked by selects.
        double vc = 0.0, dot = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
          const int i = part + 8 * k;
          const double v = vcol[b][i];
          vc = (i == c) ? col[k] : vc;
          dot += (i > c && i < d) ? v * col[k] : 0.0;
        }
        vc = sum8(vc);
        dot = sum8(dot);
        const double f = tau * (dot * scal + vc), fs = f * scal;
        double nxt = 0.0;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
          const int i = part + 8 * k;
          const double v = vcol[b][i];
          const double upd = (i > c && i < d) ? col[k] - fs * v : (i == c ? col[k] - f : col[k]);
          col[k] = upd;
          nxt += (i >= c + 2 && i < d) ? upd * upd : 0.0;
        }
        if (q == c + 1) {  // publish the next reflector column and its tail norm
#pragma unroll
          for (int k = 0; k < KR; ++k) vcol[b ^ 1][part + 8 * k] = col[k];
          nxt = sum8(nxt);
          if (part == 0) tail2[c + 1] = nxt;
        }
      }
    }
    __syncthreads();
    // T = upper triangle of the factor with a positive diagonal (appendix: sign of t_11)
    if (q < cols) {
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int i = part + 8 * k;
        if (i < q) Ts[i * ldT + q] = (diagR[i] < 0.0) ? -col[k] : col[k];
      }
    }
    for (int i = tid; i < cols; i += kWhitenThreads) Ts[i * ldT + i] = fabs(diagR[i]);
  } else {
    for (int i = tid; i < cols; i += kWhitenThreads) Ts[i * ldT + i] = 1.0;
  }
  __syncthreads();
  whiten_tail(a, Ts, ldT, mm, brk, s_lds);
  if (tid == 0) st->whiten_chol = 0;
}

// Whitening QR for large d (> 512): the same column-parallel Householder QR with the basis in
// global scratch (U copied to a.Uq).
__global__ __launch_bounds__(kWhitenThreads) void k_whiten_mem(SmallArgs a0) {
  __shared__ double Ts[(kMaxM + 1) * (kMaxM + 1)];
  __shared__ double rfs[2][2];
  __shared__ double diagR[kMaxM + 1];
  __shared__ double tail2[kMaxM + 2];
  __shared__ double s_lds[kMaxM];
  const SmallArgs a = member_args(a0);
  State* st = a.st;
  if (st->done) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int d = a.d;
  const int mm = st->meff;
  const int brk = st->brk;
  if (st->nonfinite || mm == 0) return;
  const int cols = brk ? mm : mm + 1;
  const int ldT = kMaxM + 1;
  for (int e = tid; e < cols * cols; e += kWhitenThreads) Ts[(e / cols) * ldT + (e % cols)] = 0.0;
  __syncthreads();  // the zeros land before any entry of T is written below
  if (!a.plain) {
    double* Ub = a.Uq;
    for (int e = tid; e < d * cols; e += kWhitenThreads) Ub[e] = a.U[e];
    const int q = wv * 8 + (lane >> 3), part = lane & 7;
    double* uq = Ub + (size_t)q * d;
    __syncthreads();
    if (q == 0) {
      double s0 = 0.0;
      for (int i = 1 + part; i < d; i += 8) s0 += uq[i] * uq[i];
      s0 = sum8(s0);
      if (part == 0) tail2[0] = s0;
    }
    for (int c = 0; c < cols; ++c) {
      const double* uc = Ub + (size_t)c * d;
      const int b = c & 1;
      if (q == c && part == 0) {
        const double s2 = tail2[c];
        const double alp = uc[c];
        const double nrm = sqrt(alp * alp + s2);
        double tau = 0.0, beta_h = alp, scal = 0.0;
        if (s2 > 0.0 || alp < 0.0) {
          beta_h = (alp >= 0.0) ? -nrm : nrm;
          tau = (beta_h - alp) / beta_h;
          scal = 1.0 / (alp - beta_h);
        }
        rfs[b][0] = tau;
        rfs[b][1] = scal;
        diagR[c] = beta_h;
      }
      __syncthreads();
      const double tau = rfs[b][0], scal = rfs[b][1];
      if (q > c && q < cols) {
        double nxt = 0.0;
        if (tau != 0.0) {
          double dot = 0.0;
          for (int i = c + 1 + part; i < d; i += 8) dot += uc[i] * uq[i];
          dot = sum8(dot);
          const double f = tau * (dot * scal + uq[c]);
          const double fs = f * scal;
          for (int i = c + 1 + part; i < d; i += 8) {
            const double v = uq[i] - fs * uc[i];
            uq[i] = v;
            if (i >= c + 2) nxt += v * v;
          }
          if (part == 0) uq[c] -= f;
        } else if (q == c + 1) {
          for (int i = c + 2 + part; i < d; i += 8) nxt += uq[i] * uq[i];
        }
        if (q == c + 1) {
          nxt = sum8(nxt);
          if (part == 0) tail2[c + 1] = nxt;
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < cols * cols; e += kWhitenThreads) {
      const int i = e / cols, l = e % cols;
      if (l > i) Ts[i * ldT + l] = (diagR[i] < 0.0) ? -Ub[(size_t)l * d + i] : Ub[(size_t)l * d + i];
      else if (l == i) Ts[i * ldT + l] = fabs(diagR[i]);
    }
  } else {
    for (int i = tid; i < cols; i += kWhitenThreads) Ts[i * ldT + i] = 1.0;
  }
  __syncthreads();
  whiten_tail(a, Ts, ldT, mm, brk, s_lds);
  if (tid == 0) st->whiten_chol = 0;
}

// Quadrature solves, one wavefront per system s: (zeta_s I - Rt) y = e_1 with Rt upper Hessenberg.
// Lane l holds column l of the row being eliminated (m <= 64); Gaussian elimination with partial
// pivoting between neighbouring rows stores the triangular factor in LDS, then a column-oriented
// back substitution needs one broadcast per row.  Stores its term alpha w_s psi_s y of the pass
// coefficients in row s of the g buffer (k_combine adds the rows of a time point in node order)
// and advances psi_s <- psi_s alpha r tau y_m.
// v of lane src (src the same in every lane), through the scalar unit rather than an LDS permute
__device__ __forceinline__ cplx bcast_c(cplx v, int src) { return cplx{bcast_lane(v.re, src), bcast_lane(v.im, src)}; }
// 1 / b through one real division (the moduli met here are far from the FP64 range limits)
__device__ __forceinline__ cplx crecip(cplx b) {
  const double s = 1.0 / (b.re * b.re + b.im * b.im);
  return cplx{b.re * s, -b.im * s};
}

__global__ __launch_bounds__(64) void k_quad(SmallArgs a0) {
  extern __shared__ unsigned char smq[];
  const SmallArgs a = member_args(a0);
  const State* st = a.st;
  const int mm = st->meff;
  if (st->done || st->nonfinite || mm == 0) return;
  const int ld = mm + 1;
  double* Xs = reinterpret_cast<double*>(smq);
  cplx* Us = reinterpret_cast<cplx*>(smq + (((size_t)mm * ld * 8 + 15) & ~(size_t)15));
  const int sidx = blockIdx.x, lane = threadIdx.x;
  // Rt (m x m column-major in global memory, written by the previous kernel) into LDS, row-major:
  // lane i takes row i, sixteen columns per round trip (one load per trip costs a memory latency
  // per column)
  for (int l0 = 0; l0 < mm; l0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = (lane < mm && l0 + u < mm) ? a.Xout[(size_t)(l0 + u) * a.m + lane] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (lane < mm && l0 + u < mm) Xs[lane * ld + l0 + u] = v[u];
  }
  __syncthreads();
  const cplx zeta = a.rz[sidx];
  auto H = [&](int i, int l) -> cplx {
    const double x = Xs[i * ld + l];
    return (i == l) ? cmk(zeta.re - x, zeta.im) : cmk(-x, 0.0);
  };
  cplx carry = (lane < mm) ? H(0, lane) : cmk(0.0, 0.0);
  cplx rc = cmk(1.0, 0.0);
  cplx r = cmk(0.0, 0.0);  // right-hand side entry of row `lane` after elimination
  for (int i = 0; i < mm - 1; ++i) {
    const cplx av = bcast_c(carry, i);
    const cplx hb = (lane < mm) ? H(i + 1, lane) : cmk(0.0, 0.0);
    const cplx bs = bcast_c(hb, i);
    if (cabs1(bs) > cabs1(av)) {  // pivot on row i+1 (uniform branch)
      const cplx mult = cmul(av, crecip(bs));
      if (lane >= i && lane < mm) Us[i * ld + lane] = hb;
      if (lane == i) r = cmk(0.0, 0.0);
      carry = csub(carry, cmul(mult, hb));
    } else {
      const cplx mult = (av.re == 0.0 && av.im == 0.0) ? cmk(0.0, 0.0) : cmul(bs, crecip(av));
      if (lane >= i && lane < mm) Us[i * ld + lane] = carry;
      if (lane == i) r = rc;
      carry = csub(hb, cmul(mult, carry));
      rc = csub(cmk(0.0, 0.0), cmul(mult, rc));
    }
  }
  if (lane == mm - 1) {
    Us[(mm - 1) * ld + lane] = carry;
    r = rc;
  }
  __syncthreads();
  const cplx inv_ll = (lane < mm) ? crecip(Us[lane * ld + lane]) : cmk(0.0, 0.0);
  cplx y = cmk(0.0, 0.0);
  for (int i = mm - 1; i >= 0; --i) {
    const cplx yi = cmul(bcast_c(r, i), bcast_c(inv_ll, i));
    if (lane == i) y = yi;
    if (lane < i) r = csub(r, cmul(Us[lane * ld + i], yi));
  }
  const cplx ps = a.psi[sidx];
  const cplx wp = cmul(a.rw[sidx], ps);
  {
    // this node's term alpha * w psi y of its time point's coefficients (twice the real part for the
    // conjugate-half rules)
    const double fac = rule_is_half(a.fun) ? 2.0 : 1.0;
    if (lane < mm) a.gbuf[(size_t)sidx * a.m + lane] = fac * st->alpha * cmul(wp, y).re;
  }
  const cplx ym = bcast_c(y, mm - 1);
  if (lane == 0) a.psi[sidx] = cscale(cmul(ps, ym), st->cpl);
}

// Pass coefficients C[:, t] (t < nt): the rule nodes' terms of each time point added in node order
// (a fixed order, so the same bits on every run); the restart column C[:, nt] was written by the
// whitening kernel.
__global__ __launch_bounds__(kThreads) void k_combine(SmallArgs a0) {
  const SmallArgs a = member_args(a0);
  const State* st = a.st;
  if (st->done) return;
  const int m = a.m, nt = a.nt, mm = st->meff, nq = a.nq;
  const bool zero = st->nonfinite || mm == 0;
  for (int e = threadIdx.x; e < (m + 1) * nt; e += kThreads) {
    const int i = e % (m + 1), it = e / (m + 1);
    double v = 0.0;
    if (!zero && i < mm) {  // eight loads in flight, added in node order
      const double* g = a.gbuf + (size_t)it * nq * m + i;
      int l = 0;
      for (; l + 8 <= nq; l += 8) {
        double t8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t8[u] = g[(size_t)(l + u) * m];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t8[u];
      }
      for (; l < nq; ++l) v += g[(size_t)l * m];
    }
    a.C[e] = v;
  }
  if (zero)
    for (int i = threadIdx.x; i <= m; i += kThreads) a.C[(size_t)nt * (m + 1) + i] = 0.0;
}

// ------------------------------------------------------------------------ growing restart
// The restart of Algorithm 2 as the paper states it: f applied to the growing block matrix of all
// cycles so far, instead of the fixed-size quadrature recursion.  In the basis the cycle end uses
// (Rt = T_m^{-1} X T_m per cycle, the similarity above), that matrix is upper Hessenberg: diagonal
// blocks Rt_1 .. Rt_c and, between cycles c-1 and c, the single entry r tau alpha_c in the first row
// of block c and the last column of block c-1 (X's coupling h beta_c = r tau alpha_c T_11 / T_mm
// carried through the two diagonal similarities).  With beta_1 = alpha_1 T_11 the pass coefficients
// of cycle c are then c_t = alpha_1 [f(M_c) e_1] restricted to block c.  f = exp(-t z) only.
//
// Storage: block c (size sz_c <= m) column-major with leading dimension m at gM + m * (rows of
// blocks 1..c-1); gK[c] its coupling to block c-1; gSz[c] its size.

// One block: append this cycle's Rt and coupling.
__global__ __launch_bounds__(kThreads) void k_grow_append(SmallArgs a, double* __restrict__ gM,
                                                          double* __restrict__ gK, int* __restrict__ gSz) {
  State* st = a.st;
  if (st->done) return;
  const int m = a.m, mm = st->meff;
  if (st->nonfinite || mm == 0) return;
  const int c = st->grow_c, p = st->grow_p;
  if (p + mm > kGrowRows) {  // capacity (the host keeps max_cycles * m within it)
    if (threadIdx.x == 0) st->grow_fail = 1;
    return;
  }
  double* blk = gM + (size_t)p * m;
  for (int e = threadIdx.x; e < mm * mm; e += kThreads) {
    const int i = e % mm, j = e / mm;
    blk[i + (size_t)j * m] = a.Xout[i + (size_t)j * m];
  }
  if (threadIdx.x == 0) {
    gK[c] = (c == 0) ? 0.0 : st->grow_rt * st->alpha;
    gSz[c] = mm;
    if (c == 0) st->grow_alpha1 = st->alpha;
    st->grow_rt = st->brk ? 0.0 : st->cpl / st->alpha;  // cpl = alpha r tau, alpha > 0 here
    st->grow_c = c + 1;
    st->grow_p = p + mm;
  }
}

// exp(-t M) e_1 for the time point t = tvals[blockIdx.x] by the truncated Taylor series applied to a
// vector (Al-Mohy and Higham 2011, the action of the matrix exponential): s steps of
// v <- sum_{k <= K} (B^k / k!) v with B = -t M / s.  s = ceil(t ||M||_1 / 2), so ||B||_1 <= 2, and K
// is the first degree whose next term bound eta^(K+1) / (K+1)! (eta = ||B||_1) is below 2^-53.
// One thread per row of M (rows <= kGrowRows); the vector is in LDS.  Writes the pass
// coefficients of the current cycle (column blockIdx.x of C), zeros past the basis.
__global__ __launch_bounds__(kGrowRows) void k_grow_expmv(SmallArgs a, const double* __restrict__ gM,
                                                          const double* __restrict__ gK,
                                                          const int* __restrict__ gSz,
                                                          const double* __restrict__ tvals) {
  __shared__ double tv[kGrowRows];
  __shared__ double colsum[kGrowRows];
  __shared__ double red[kGrowRows / 64];
  State* st = a.st;
  if (st->done) return;
  const int m = a.m, it = blockIdx.x, i = threadIdx.x;
  double* Ccol = a.C + (size_t)it * (m + 1);
  const int mm = st->meff;
  if (st->nonfinite || mm == 0 || st->grow_fail) {
    for (int e = i; e <= m; e += kGrowRows) Ccol[e] = 0.0;
    if (it == 0)
      for (int e = i; e <= m; e += kGrowRows) a.C[(size_t)a.nt * (m + 1) + e] = 0.0;
    return;
  }
  const int p = st->grow_p;
  // this thread's row: block c, local row li, first row of the block off
  int c = 0, off = 0;
  if (i < p)
    while (off + gSz[c] <= i) off += gSz[c++];
  const int li = i - off, sz = (i < p) ? gSz[c] : 0;
  const double* blk = gM + (size_t)off * m;
  const int j0 = li > 0 ? li - 1 : 0;  // Hessenberg: entries from column li - 1 on
  const double kap = (i < p && li == 0 && c > 0) ? gK[c] : 0.0;
  // ||M||_1: thread i sums column i (blocks are square, so column i is local column li of block c):
  // rows 0 .. li+1 of its block (Hessenberg) and, for a block's last column, the coupling entry
  // in the first row of the next block; each sum in row order
  if (i < p) {
    double cs = 0.0;
    const int rmax = min(li + 1, sz - 1);
    for (int r = 0; r <= rmax; ++r) cs += fabs(blk[r + (size_t)li * m]);
    if (li == sz - 1 && c + 1 < st->grow_c) cs += fabs(gK[c + 1]);
    colsum[i] = cs;
  }
  __syncthreads();
  double cmax = 0.0;
  for (int e = i; e < p; e += kGrowRows) cmax = fmax(cmax, colsum[e]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
  if ((i & 63) == 0) red[i >> 6] = cmax;
  __syncthreads();
  cmax = 0.0;
  for (int q = 0; q < kGrowRows / 64; ++q) cmax = fmax(cmax, red[q]);
  const double t = tvals[it];
  const double anorm = t * cmax;
  const double sd = fmax(1.0, ceil(anorm / 2.0));
  if (!(sd <= (double)kGrowMaxSteps)) {  // also catches a non-finite norm
    if (i == 0) st->grow_fail = 1;
    for (int e = i; e <= m; e += kGrowRows) Ccol[e] = 0.0;
    return;
  }
  const int steps = (int)sd;
  const double eta = anorm / sd, scale = -t / sd;
  int K = 1;  // first degree with eta^(K+1) / (K+1)! < 2^-53 (uniform over the block)
  {
    double b = eta;  // eta^k / k! at k = K
    while (K < 60 && b * eta / (K + 1) >= 1.1102230246251565e-16) {
      b = b * eta / (K + 1);
      ++K;
    }
  }
  double acc = (i == 0) ? 1.0 : 0.0;  // v = e_1
  for (int sstep = 0; sstep < steps; ++sstep) {
    __syncthreads();  // the previous step's readers of tv are done
    if (i < p) tv[i] = acc;
    double term = acc;
    for (int k = 1; k <= K; ++k) {
      __syncthreads();  // tv holds the previous term
      double y = 0.0;
      if (i < p) {
        for (int jj = j0; jj < sz; ++jj) y = fma(blk[li + (size_t)jj * m], tv[off + jj], y);
        if (kap != 0.0) y = fma(kap, tv[off - 1], y);
      }
      term = y * (scale / (double)k);
      __syncthreads();  // every row has read the previous term
      if (i < p) tv[i] = term;
      acc += term;
    }
  }
  // coefficients of the current (last) block
  const int lastoff = p - mm;
  const double a1 = st->grow_alpha1;
  if (i >= lastoff && i < p) Ccol[i - lastoff] = a1 * acc;
  for (int e = mm + i; e <= m; e += kGrowRows) Ccol[e] = 0.0;
}

hipError_t launch_small_grow(hipStream_t s, const SmallArgs& a, double* gM, double* gK, int* gSz,
                             const double* tvals) {
  hipLaunchKernelGGL(k_grow_append, dim3(1), dim3(kThreads), 0, s, a, gM, gK, gSz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grow_expmv, dim3(a.nt), dim3(kGrowRows), 0, s, a, gM, gK, gSz, tvals);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------ fused pass
// x_t += W c_t for every time point, v_hat = W c_nt written over column 0, and per-block partial
// norms ||y_t||^2, ||x_t||^2, written to entries dn + 2t and dn + 2t + 1 of the partial buffer
// (k_reduce_parts adds the blocks in a fixed order).
constexpr int kPassGroup = 8;  // basis columns whose loads the pass issues together

// With ps.on, the pass also sketches v_hat for the next cycle's start (alpha = ||S v_hat||,
// u_1 = S v_hat / alpha): each row's S column is regenerated as in the fused product and added
// into d bins in LDS (one set per wavefront, as there), whose fixed-order sums go to entries
// [0, d) of the partial buffer.  That spares the next cycle a sketch-only pass over v_hat; the
// extra ALU work hides under the pass's loads.
template <typename T, int NT>
__global__ __launch_bounds__(kThreads) void k_pass(int n, int m, int nt, int dn, const double* __restrict__ C,
                                                   T* __restrict__ W, double* __restrict__ x, int64_t ldx,
                                                   double* __restrict__ parts, const State* __restrict__ st,
                                                   size_t bs, PassSketch ps) {
  // From four time points on, the weights C (nt + 1 per basis column) outgrow the scalar registers:
  // the compiler then spills them to vector lanes and reads them back with one VALU instruction per
  // word (k_pass<float, 8>: 1.8e9 VALU instructions per launch on the batched 1024^2 workload).  So
  // they go to LDS once per block instead, a row of kCs per column, read by broadcast (that pass:
  // 3.95 -> 2.99 ms per launch, same bits).
  constexpr bool kLdsC = NT >= 4;
  constexpr int kCs = (NT + 2) & ~1;  // q = 0 .. NT - 1 time points, q = NT the restart, then 0
  __shared__ double sC[kLdsC ? (kMaxM + 1) * kCs : 1];
  __shared__ double part[kThreads / 64][2 * NT];
  extern __shared__ double pbins[];  // (kThreads / 64) x ps.d bins when sketching
  st = bat(st, bs);
  const int mm = st->meff;
  if (st->done || st->nonfinite || mm == 0) return;
  C = bat(C, bs);
  W = bat(W, bs);
  parts = bat(parts, bs);
  x += (int64_t)blockIdx.y * nt * ldx;  // member r's time points are columns r nt .. r nt + nt - 1
  const int brk = st->brk;
  const int ncol = brk ? mm : mm + 1;
  const bool sk = ps.on && !brk;  // block-uniform
  double* wbins = pbins + (threadIdx.x >> 6) * ps.d;
  if (sk)
    for (int b = threadIdx.x; b < (kThreads / 64) * ps.d; b += kThreads) pbins[b] = 0.0;
  if constexpr (kLdsC)
    for (int e = threadIdx.x; e < ncol * kCs; e += kThreads) {
      const int j = e / kCs, q = e % kCs;
      sC[e] = q < nt ? C[(size_t)q * (m + 1) + j] : (q == NT ? C[(size_t)nt * (m + 1) + j] : 0.0);
    }
  if (sk || kLdsC) __syncthreads();
  double yn[NT], xn[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) yn[q] = xn[q] = 0.0;
  const size_t ld = wcol(n, sizeof(T));
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < (size_t)n; i += stride) {
    double acc[NT + 1];
#pragma unroll
    for (int q = 0; q <= NT; ++q) acc[q] = 0.0;
    // columns in groups of kPassGroup: all loads of a group are issued before its products (past
    // the last column the index is clamped and the weight is 0, so no load is guarded); the
    // basis is not read again before the next cycle overwrites it, hence non-temporal loads.  The
    // weights C (time point q, basis index j) have addresses uniform over the block, so they come
    // through scalar loads, not one LDS read per product (2.4% of the pass)
    for (int j0 = 0; j0 < ncol; j0 += kPassGroup) {
      T wv[kPassGroup];
#pragma unroll
      for (int u = 0; u < kPassGroup; ++u)
        wv[u] = __builtin_nontemporal_load(&W[(size_t)min(j0 + u, ncol - 1) * ld + i]);
#pragma unroll
      for (int u = 0; u < kPassGroup; ++u) {
        const int j = min(j0 + u, ncol - 1);
        const double w = (j0 + u < ncol) ? (double)wv[u] : 0.0;
#pragma unroll
        for (int q = 0; q <= NT; ++q) {  // q = NT: the restart column, stored after the nt time points
          double cq;
          if constexpr (kLdsC) cq = sC[j * kCs + q];
          else cq = (q < nt) ? C[(size_t)q * (m + 1) + j] : (q == NT ? C[(size_t)nt * (m + 1) + j] : 0.0);
          acc[q] = fma(w, cq, acc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (q < nt) {
        double* xp = x + (size_t)q * ldx + i;
        const double xv = *xp + acc[q];
        *xp = xv;
        yn[q] += acc[q] * acc[q];
        xn[q] += xv * xv;
      }
    }
    if (!brk) W[i] = (T)acc[NT];
    if (sk) {
      int rows[8];
      uint32_t sb = 0;
      sketch_column<8>((uint64_t)i, ps.d, ps.zeta, ps.k0, ps.k1, rows, sb);
      const double zs = (double)(T)acc[NT] * ps.scale;  // the stored value, as the next cycle reads it
#pragma unroll
      for (int l = 0; l < 8; ++l)
        if (l < ps.zeta) unsafeAtomicAdd(&wbins[rows[l]], ((sb >> l) & 1u) ? -zs : zs);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const double a1 = wave_sum_c(yn[q]), a2 = wave_sum_c(xn[q]);
    if (lane == 0) {
      part[wv][2 * q] = a1;
      part[wv][2 * q + 1] = a2;
    }
  }
  __syncthreads();
  const size_t pidx = part_index();
  if (threadIdx.x < 2 * nt) {
    double s = part[0][threadIdx.x];
    for (int q = 1; q < kThreads / 64; ++q) s += part[q][threadIdx.x];
    parts[(size_t)(dn + threadIdx.x) * kMaxParts + pidx] = s;
  }
  if (ps.on) {  // the barrier above ordered every bin update before these reads; zeros after a breakdown
    for (int b = threadIdx.x; b < ps.d; b += kThreads) {
      double v = 0.0;
      if (sk) {
        v = pbins[b];
        for (int q = 1; q < kThreads / 64; ++q) v += pbins[q * ps.d + b];
      }
      parts[(size_t)b * kMaxParts + pidx] = v;
    }
  }
}

// Convergence test after the pass: the error estimate after Algorithm 2 (the difference of two
// successive cycles, y_c = x_c - x_{c-1}) read as the first of the remaining increments.  With q
// the largest of the last three contraction ratios ||y_c|| / ||y_{c-1}|| of a time point (fewer in
// cycles 2 and 3), the remaining error is estimated by the geometric tail
//   err_t = (||y_c|| / ||x_c||) q / (1 - q)   for q < 1, and is unbounded for q >= 1
// (in particular after the first cycle, which has no ratio).  Small ratios between growing
// increments (a dip inside a transient) do not end the loop.  A time point whose relative
// increment is at or below the unit roundoff of the value type (uround) is converged, err_t being
// the increment itself: there the increments are rounding noise whose ratios scatter around 1, and
// a point that converged early (a small t) would otherwise hold back the others.  The time points
// share one Krylov basis (the restart vector does not depend on t), so each point's estimates are
// those of its own single solve; a point that has passed (err_t <= tol) is not tested again and
// keeps the estimate it passed with, and the solve stops in the cycle in which the last point
// passes, the largest of the single solves' cycle counts.  The solve stops when
// max_t err_t <= tol.  The raw relative increment max_t ||y_c|| / ||x_c|| is reported too; it
// decides divergence.  The norms are the fixed-order sums of the pass's partials (red + dn).
__global__ void k_final(int nt, int dn, double tol, double div_limit, double uround, const double* __restrict__ red,
                        State* __restrict__ st, Report* __restrict__ rep, size_t bs) {
  if (threadIdx.x != 0) return;
  st = bat(st, bs);
  red = bat(red, bs) + dn;
  rep += blockIdx.y;
  if (st->done) {  // finished in an earlier cycle: report unchanged
    rep->done = 1;
    return;
  }
  const double inf = __builtin_inf();
  const int c = st->cyc;
  double est = 0.0, rel = 0.0, qd = 0.0;
  for (int it = 0; it < nt; ++it) {
    const double y2 = red[2 * it], x2 = red[2 * it + 1];
    st->ynorm2[it] = y2;
    st->xnorm2[it] = x2;
    const double y = sqrt(y2);
    const double r = (x2 > 0.0) ? sqrt(y2 / x2) : 0.0;
    rel = fmax(rel, r);
    const double yp = st->yprev[it];
    const double q = (c == 0) ? inf : (yp > 0.0 ? y / yp : (y > 0.0 ? inf : 0.0));
    double qb = q;
    if (c >= 2) qb = fmax(qb, st->qprev[it]);
    if (c >= 3) qb = fmax(qb, st->qprev2[it]);
    // an increment at the unit roundoff of the value type is rounding noise: its own estimate
    double e = (r <= uround) ? r : (qb < 1.0 ? r * qb / (1.0 - qb) : inf);
    if ((st->passed_mask >> it) & 1) {
      e = st->passed[it];  // passed in an earlier cycle: no longer tested
    } else if (e <= tol) {
      st->passed_mask |= 1 << it;
      st->passed[it] = e;
    }
    est = fmax(est, e);
    st->yprev[it] = y;
    st->qprev2[it] = st->qprev[it];
    st->qprev[it] = q;
  }
  st->cyc = c + 1;
  st->relupd = rel;
  qd = st->rule_err;
  st->est = est;
  st->converged = (est <= tol) ? 1 : 0;
  rep->est = est;
  rep->relupd = rel;
  rep->rule_err = qd;
  rep->alpha = st->alpha;
  rep->beta = st->beta;
  rep->kappa_T = st->kappa_T;
  rep->brk = st->brk;
  rep->meff = st->meff;
  rep->nonfinite = st->nonfinite;
  rep->converged = st->converged;
  rep->grow_fail = st->grow_fail;
  st->done = (st->converged || st->brk || st->nonfinite || !(rel <= div_limit)) ? 1 : 0;
  rep->done = st->done;
}

// Rows and signs of S for a range of columns (specification test hook).
template <int ZMAX>
__global__ void k_sketch_table(int64_t col0, int64_t count, int d, int zeta, uint32_t k0, uint32_t k1,
                               int* __restrict__ rows_out, int8_t* __restrict__ signs_out) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < count; c += (int64_t)gridDim.x * blockDim.x) {
    int rows[ZMAX];
    uint32_t sb;
    sketch_column<ZMAX>((uint64_t)(col0 + c), d, zeta, k0, k1, rows, sb);
#pragma unroll
    for (int l = 0; l < ZMAX; ++l) {
      if (l < zeta) {
        rows_out[c * zeta + l] = rows[l];
        signs_out[c * zeta + l] = ((sb >> l) & 1u) ? (int8_t)-1 : (int8_t)1;
      }
    }
  }
}

// FP64 dot product <x, y> with a fixed summation order (per-block partials, then one block):
// the same grid gives the same bits on every call.
__global__ __launch_bounds__(kThreads) void k_dot_partial(int64_t n, const double* __restrict__ x,
                                                          const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double buf[kThreads / 64];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) acc = fma(x[i], y[i], acc);
  acc = wave_sum_c(acc);
  if ((threadIdx.x & 63) == 0) buf[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += buf[q];
    part[blockIdx.x] = s;
  }
}

__global__ void k_dot_final(int nb, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    *out = s;
  }
}

// ------------------------------------------------------------------------------------ launchers
hipError_t launch_zero_strided(hipStream_t s, double* p, size_t count, int reps, size_t step_bytes) {
  if (count == 0 || reps == 0) return hipSuccess;
  int grid = (int)((count + 255) / 256);
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(k_zero_strided, dim3(grid, reps), dim3(256), 0, s, p, count, step_bytes);
  return hipGetLastError();
}

hipError_t launch_zero(hipStream_t s, double* p, size_t count) {
  if (count == 0) return hipSuccess;
  int grid = (int)((count + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_rule(hipStream_t s, int fun, int nt, const double* tvals, int n_main, double lo, double hi,
                       cplx* rz, cplx* rw, cplx* psi, State* st, int nb, size_t bs) {
  hipLaunchKernelGGL(k_rule, dim3(8, nb), dim3(256), 0, s, fun, nt, tvals, n_main, lo, hi, rz, rw, psi, bs);
  const int nq = rule_is_half(fun) ? n_main / 2 : n_main;
  hipLaunchKernelGGL(k_rule_check, dim3(1), dim3(kRuleSamples), 0, s, fun, nt, tvals, nq, lo, hi, rz, rw, st, nb,
                     bs);
  return hipGetLastError();
}

hipError_t launch_copy_in(hipStream_t s, int dtype, int grid, int n, const void* b, int64_t ldb, void* w0, int nb,
                          size_t bs) {
  const dim3 g(grid, nb);
  if (dtype == 0)
    hipLaunchKernelGGL(k_copy_in<double>, g, dim3(256), 0, s, n, (const double*)b, ldb, (double*)w0, bs);
  else
    hipLaunchKernelGGL(k_copy_in<float>, g, dim3(256), 0, s, n, (const float*)b, ldb, (float*)w0, bs);
  return hipGetLastError();
}

hipError_t launch_sqnorm(hipStream_t s, int dtype, int grid, int n, const void* v, double* slots) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_sqnorm<double>, dim3(grid), dim3(kThreads), 0, s, n, (const double*)v, slots);
  else
    hipLaunchKernelGGL(k_sqnorm<float>, dim3(grid), dim3(kThreads), 0, s, n, (const float*)v, slots);
  return hipGetLastError();
}

hipError_t launch_start(hipStream_t s, int d, int m, int plain, const double* sv, double* slots_start,
                        double* slots_step, size_t step_len, double* U, double* R, State* st, int nb, size_t bs) {
  hipLaunchKernelGGL(k_start, dim3(1, nb), dim3(kThreads), 0, s, d, m, plain, sv, slots_start, slots_step, step_len,
                     U, R, st, bs);
  return hipGetLastError();
}

size_t quad_lds(int m) { return (size_t)m * (m + 1) * 8 + 16 + (size_t)m * (m + 1) * sizeof(cplx); }

// The pass's bins (one set of d FP64 per wavefront) reach 128 KB at d = kMaxD.
template <typename T>
static hipError_t configure_pass_t() {
  const void* fns[] = {reinterpret_cast<const void*>(&k_pass<T, 1>), reinterpret_cast<const void*>(&k_pass<T, 2>),
                       reinterpret_cast<const void*>(&k_pass<T, 4>), reinterpret_cast<const void*>(&k_pass<T, 8>),
                       reinterpret_cast<const void*>(&k_pass<T, 16>)};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (kThreads / 64) * kMaxD * (int)sizeof(double));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t configure_cycle_kernels() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_quad),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)quad_lds(kMaxM));
  if (e == hipSuccess) e = configure_pass_t<double>();
  if (e == hipSuccess) e = configure_pass_t<float>();
  return e;
}

hipError_t launch_small_grow(hipStream_t s, const SmallArgs& a, double* gM, double* gK, int* gSz,
                             const double* tvals);

// The cycle end of every batch member (a.bs apart): whitening, then the restart coefficients, by
// the quadrature recursion or (grow given; one member) by the growing block matrix.
hipError_t launch_small(hipStream_t s, const SmallArgs& a, int nb, const GrowBuffers* grow) {
  const dim3 g1(1, nb);
  if (a.plain || a.d <= 64)
    hipLaunchKernelGGL(k_whiten<8>, g1, dim3(kWhitenThreads), 0, s, a);
  else if (a.d <= 200)  // 25 rows per lane: no idle register rows at d = 200
    hipLaunchKernelGGL(k_whiten<25>, g1, dim3(kWhitenThreads), 0, s, a);
  else if (a.d <= 256)
    hipLaunchKernelGGL(k_whiten<32>, g1, dim3(kWhitenThreads), 0, s, a);
  else if (a.d <= 512)
    hipLaunchKernelGGL(k_whiten<64>, g1, dim3(kWhitenThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_whiten_mem, g1, dim3(kWhitenThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (grow) return launch_small_grow(s, a, grow->M, grow->K, grow->sz, grow->tvals);
  const int nsys = a.nt * a.nq;
  hipLaunchKernelGGL(k_quad, dim3(nsys, nb), dim3(64), quad_lds(a.m), s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_combine, g1, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
static void launch_pass_t(hipStream_t s, int grid, int n, int m, int nt, int dn, const double* C, T* W, double* x,
                          int64_t ldx, double* parts, const State* st, int nb, size_t bs, const PassSketch& ps) {
  const dim3 g(grid, nb);
  const size_t lds = ps.on ? (size_t)(kThreads / 64) * ps.d * sizeof(double) : 0;
#define FAB_P(NTV) \
  hipLaunchKernelGGL((k_pass<T, NTV>), g, dim3(kThreads), lds, s, n, m, nt, dn, C, W, x, ldx, parts, st, bs, ps)
  if (nt <= 1)
    FAB_P(1);
  else if (nt <= 2)
    FAB_P(2);
  else if (nt <= 4)
    FAB_P(4);
  else if (nt <= 8)
    FAB_P(8);
  else
    FAB_P(16);
#undef FAB_P
}

hipError_t launch_pass(hipStream_t s, int dtype, int grid, int n, int m, int nt, int dn, const double* C, void* W,
                       double* x, int64_t ldx, double* parts, const State* st, int nb, size_t bs,
                       const PassSketch& ps) {
  if (ps.on && (ps.zeta < 1 || ps.zeta > 8 || ps.d < 1 || ps.d > kMaxD || ps.d != dn)) return hipErrorInvalidValue;
  if (grid < kXcds || grid > kMaxParts || grid % kXcds != 0) return hipErrorInvalidValue;  // part_index
  if (dtype == 0)
    launch_pass_t<double>(s, grid, n, m, nt, dn, C, (double*)W, x, ldx, parts, st, nb, bs, ps);
  else
    launch_pass_t<float>(s, grid, n, m, nt, dn, C, (float*)W, x, ldx, parts, st, nb, bs, ps);
  return hipGetLastError();
}

hipError_t launch_final(hipStream_t s, int nt, int dn, double tol, double div_limit, double uround, const double* red,
                        State* st, Report* rep, int nb, size_t bs) {
  hipLaunchKernelGGL(k_final, dim3(1, nb), dim3(64), 0, s, nt, dn, tol, div_limit, uround, red, st, rep, bs);
  return hipGetLastError();
}

hipError_t launch_sketch_table(hipStream_t s, int64_t col0, int64_t count, int d, int zeta, uint64_t seed,
                               int* rows, int8_t* signs) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  int grid = (int)((count + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (grid < 1) grid = 1;
  if (zeta <= 1)
    hipLaunchKernelGGL(k_sketch_table<1>, dim3(grid), dim3(256), 0, s, col0, count, d, zeta, k0, k1, rows, signs);
  else if (zeta <= 4)
    hipLaunchKernelGGL(k_sketch_table<4>, dim3(grid), dim3(256), 0, s, col0, count, d, zeta, k0, k1, rows, signs);
  else if (zeta <= 8)
    hipLaunchKernelGGL(k_sketch_table<8>, dim3(grid), dim3(256), 0, s, col0, count, d, zeta, k0, k1, rows, signs);
  else if (zeta <= 16)
    hipLaunchKernelGGL(k_sketch_table<16>, dim3(grid), dim3(256), 0, s, col0, count, d, zeta, k0, k1, rows, signs);
  else
    hipLaunchKernelGGL(k_sketch_table<32>, dim3(grid), dim3(256), 0, s, col0, count, d, zeta, k0, k1, rows, signs);
  return hipGetLastError();
}

hipError_t launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* part, int max_blocks,
                      double* out) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > max_blocks) g = max_blocks;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_dot_partial, dim3((int)g), dim3(kThreads), 0, s, n, x, y, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(64), 0, s, (int)g, part, out);
  return hipGetLastError();
}
}  // namespace fab
