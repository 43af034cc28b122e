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
#include "fab_internal.h"

namespace fab {

__device__ __forceinline__ double wave_sum_c(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Fill a double buffer with zeros (used instead of memset so the same code can sit in a graph).
__global__ void k_zero(double* p, size_t count) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

// ------------------------------------------------------------------------------- quadrature rules
// fun 0, exp(-t z): parabolic Hankel contour s(u) = P - mu u^2 + 2 i mu u, u in [-U, U],
//   U = sqrt((P+L)/mu), N midpoint nodes; zeta = -s/t, w = -h s'(u) e^s / (2 pi i t).  Only the
//   nodes with u < 0 (Im zeta > 0) are kept: for real X the other half are conjugates, and the
//   accumulation takes twice the real part.  Main rule (N, 3, 6, 45), check rule (3N/4, 5, 8, 45).
// fun 1, z^(-1/2) = (2/pi) int_0^inf (z + s^2)^{-1} ds with s = c tan(theta), N midpoint nodes on
//   (0, pi/2): zeta = -c^2 tan^2(theta), w = -(c/N) sec^2(theta), c = (lo hi)^(1/4).  Check rule 3N/4.
// Layout per time point t: nq_main main nodes then nq_chk check nodes (nq_tot = nq_main + nq_chk).
__global__ void k_rule(int fun, int nt, const double* __restrict__ tvals, int n_main, double lo, double hi,
                       cplx* __restrict__ rz, cplx* __restrict__ rw, cplx* __restrict__ psi) {
  const int n_chk = (3 * n_main) / 4;
  const int nq_main = (fun == 0) ? n_main / 2 : n_main;
  const int nq_chk = (fun == 0) ? n_chk / 2 : n_chk;
  const int nq_tot = nq_main + nq_chk;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nt * nq_tot; s += gridDim.x * blockDim.x) {
    const int it = s / nq_tot, l = s % nq_tot;
    const bool chk = l >= nq_main;
    const int idx = chk ? l - nq_main : l;
    cplx z, w;
    if (fun == 0) {
      const double t = tvals[it];
      const int N = chk ? n_chk : n_main;
      const double P = chk ? 5.0 : 3.0, mu = chk ? 8.0 : 6.0, L = 45.0;
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
    } else {
      const int N = chk ? n_chk : n_main;
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

template <typename T>
__global__ void k_copy_in(int n, const T* __restrict__ b, T* __restrict__ w0) {
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

// Cycle start (Algorithm 1, lines 1-3): alpha = ||S v|| and u_1 = S v / alpha (sketched), or
// alpha = ||v|| (plain).  Resets the per-cycle flags and zeroes all sketch accumulators.
__global__ __launch_bounds__(kThreads) void k_start(int d, int m, int plain, double* __restrict__ slots_start,
                                                    double* __restrict__ slots_step, size_t step_len,
                                                    double* __restrict__ U, double* __restrict__ R,
                                                    State* __restrict__ st) {
  __shared__ double part[kThreads / 64];
  __shared__ double s_alpha;
  double acc = 0.0;
  if (!plain) {
    for (int i = threadIdx.x; i < d; i += kThreads) {
      double s = 0.0;
      for (int c = 0; c < kSlots; ++c) s += slots_start[(size_t)c * d + i];
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
  if (!plain)
    for (int i = threadIdx.x; i < d; i += kThreads) U[i] *= inv;
  for (int i = threadIdx.x; i < kSlots * d; i += kThreads) slots_start[i] = 0.0;
  for (size_t i = threadIdx.x; i < 2 * step_len; i += kThreads) slots_step[i] = 0.0;
  for (int i = threadIdx.x; i < (m + 1) * m; i += kThreads) R[i] = 0.0;
}

// ------------------------------------------------------------------------- cycle-end small FP64


// Solve (zeta I - X) y = e_1 for upper Hessenberg X (row-major in LDS, leading dimension ldx) by
// Gaussian elimination with partial pivoting between neighbouring rows; the eliminated rows are
// kept in the system's scratch column.  Writes y (length mm) at scr[0 .. mm).
__device__ void hess_solve(int mm, const double* __restrict__ Xs, int ldx, cplx zeta, cplx* __restrict__ scr,
                           int ld) {
  // scratch regions (in elements): y [0, mm), carry [mm, 2mm), rhs [2mm, 3mm), U rows from 3mm
  auto Y = [&](int e) -> cplx& { return scr[(size_t)e * ld]; };
  auto CA = [&](int e) -> cplx& { return scr[(size_t)(mm + e) * ld]; };
  auto RH = [&](int e) -> cplx& { return scr[(size_t)(2 * mm + e) * ld]; };
  auto UR = [&](int i, int l) -> cplx& {  // row i stores columns i..mm-1
    const int off = 3 * mm + i * mm - (i * (i - 1)) / 2 + (l - i);
    return scr[(size_t)off * ld];
  };
  auto H = [&](int i, int l) -> cplx {  // (zeta I - X)[i][l]
    const double x = Xs[i * ldx + l];
    return (i == l) ? cmk(zeta.re - x, zeta.im) : cmk(-x, 0.0);
  };
  for (int l = 0; l < mm; ++l) CA(l) = H(0, l);
  cplx rc = cmk(1.0, 0.0);
  for (int i = 0; i < mm - 1; ++i) {
    const cplx a = CA(i);
    const cplx bsub = H(i + 1, i);
    if (cabs1(bsub) > cabs1(a)) {  // pivot on row i+1
      const cplx mult = cdiv(a, bsub);
      for (int l = i; l < mm; ++l) {
        const cplx hb = H(i + 1, l);
        const cplx ca = CA(l);
        UR(i, l) = hb;
        if (l > i) CA(l) = csub(ca, cmul(mult, hb));
      }
      RH(i) = cmk(0.0, 0.0);  // row i+1 has zero right-hand side; the carried rhs stays
    } else {
      const cplx mult = (a.re == 0.0 && a.im == 0.0) ? cmk(0.0, 0.0) : cdiv(bsub, a);
      for (int l = i; l < mm; ++l) {
        const cplx ca = CA(l);
        UR(i, l) = ca;
        if (l > i) CA(l) = csub(H(i + 1, l), cmul(mult, ca));
      }
      RH(i) = rc;
      rc = csub(cmk(0.0, 0.0), cmul(mult, rc));
    }
  }
  UR(mm - 1, mm - 1) = CA(mm - 1);
  RH(mm - 1) = rc;
  for (int i = mm - 1; i >= 0; --i) {
    cplx s = RH(i);
    for (int l = i + 1; l < mm; ++l) s = csub(s, cmul(UR(i, l), Y(l)));
    Y(i) = cdiv(s, UR(i, i));
  }
}

__global__ __launch_bounds__(kThreads) void k_small(SmallArgs a) {
  __shared__ double Xs[kMaxM * kMaxM];          // X row-major (also P = T R during formation)
  __shared__ double Ts[(kMaxM + 1) * (kMaxM + 1)];  // T row-major
  __shared__ double red[kThreads / 64][2];
  __shared__ double sh_scal[4];
  State* st = a.st;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = kThreads / 64;
  const int m = a.m, d = a.d, nt = a.nt;
  const int mm = st->meff;
  const int brk = st->brk;
  const int C_ld = m + 1;
  // C = 0 by default (nothing added, no restart vector)
  for (int i = tid; i < (m + 1) * (nt + 1); i += kThreads) a.C[i] = 0.0;
  if (st->nonfinite || mm == 0) return;
  const int cols = brk ? mm : mm + 1;
  const int ldT = kMaxM + 1;

  // ---- 1. T from the thin QR of U[:, :cols] (sketched) or T = I (plain Arnoldi, orthonormal basis)
  if (!a.plain) {
    for (int i = tid; i < d * cols; i += kThreads) a.Uq[i] = a.U[i];
    __syncthreads();
    for (int c = 0; c < cols; ++c) {
      double* uc = a.Uq + (size_t)c * d;
      // norm of uc[c:d] (block reduction)
      double s = 0.0;
      for (int i = c + 1 + tid; i < d; i += kThreads) s += uc[i] * uc[i];
      s = wave_sum_c(s);
      if (lane == 0) red[wv][0] = s;
      __syncthreads();
      if (tid == 0) {
        double tail = 0.0;
        for (int q = 0; q < nwv; ++q) tail += red[q][0];
        const double alp = uc[c];
        const double nrm = sqrt(alp * alp + tail);
        double tau = 0.0, beta_h = alp, scal = 0.0;
        if (tail > 0.0 || alp < 0.0) {  // reflect unless already e_c with a nonnegative entry
          beta_h = (alp >= 0.0) ? -nrm : nrm;
          tau = (beta_h - alp) / beta_h;
          scal = 1.0 / (alp - beta_h);
        }
        sh_scal[0] = tau;
        sh_scal[1] = beta_h;
        sh_scal[2] = scal;
      }
      __syncthreads();
      const double tau = sh_scal[0], beta_h = sh_scal[1], scal = sh_scal[2];
      for (int i = c + 1 + tid; i < d; i += kThreads) uc[i] *= scal;  // v = [1; uc[c+1:] * scal]
      __syncthreads();
      if (tid == 0) uc[c] = beta_h;
      // apply (I - tau v v^T) to columns c+1 .. cols-1, one wave per column
      if (tau != 0.0) {
        for (int q = c + 1 + wv; q < cols; q += nwv) {
          double* uq = a.Uq + (size_t)q * d;
          double dot = 0.0;
          for (int i = c + 1 + lane; i < d; i += 64) dot += uc[i] * uq[i];
          dot = wave_sum_c(dot) + uq[c];
          const double f = tau * dot;
          if (lane == 0) uq[c] -= f;
          for (int i = c + 1 + lane; i < d; i += 64) uq[i] -= f * uc[i];
        }
      }
      __syncthreads();
    }
    // T = upper triangle of the factor with a positive diagonal (appendix: sign of t_11)
    for (int e = tid; e < cols * cols; e += kThreads) {
      const int i = e / cols, l = e % cols;
      double v = 0.0;
      if (l >= i) {
        v = a.Uq[(size_t)l * d + i];
        if (a.Uq[(size_t)i * d + i] < 0.0) v = -v;
      }
      Ts[i * ldT + l] = v;
    }
  } else {
    for (int e = tid; e < cols * cols; e += kThreads) {
      const int i = e / cols, l = e % cols;
      Ts[i * ldT + l] = (i == l) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < (m + 1) * (m + 1); e += kThreads) {
    const int i = e % (m + 1), l = e / (m + 1);  // column-major output
    a.Tout[e] = (i < cols && l < cols) ? Ts[i * ldT + l] : 0.0;
  }

  // ---- 2. X = T_m R_m T_m^{-1} (+ rank-one), h, beta
  const double* R = a.R;
  const int ldR = m + 1;
  for (int e = tid; e < mm * mm; e += kThreads) {  // P = T_m R_m (R upper Hessenberg)
    const int i = e / mm, c = e % mm;
    double s = 0.0;
    const int lend = min(c + 1, mm - 1);
    for (int l = i; l <= lend; ++l) s += Ts[i * ldT + l] * R[(size_t)c * ldR + l];
    Xs[i * kMaxM + c] = s;
  }
  __syncthreads();
  for (int i = tid; i < mm; i += kThreads) {  // row i of X: X[i,:] T_m = P[i,:]
    for (int c = 0; c < mm; ++c) {
      double s = Xs[i * kMaxM + c];
      for (int l = 0; l < c; ++l) s -= Xs[i * kMaxM + l] * Ts[l * ldT + c];
      Xs[i * kMaxM + c] = s / Ts[c * ldT + c];
    }
  }
  __syncthreads();
  double hcoup = 0.0;
  if (!brk) {
    const double r = R[(size_t)(mm - 1) * ldR + mm];
    const double tmm = Ts[(mm - 1) * ldT + (mm - 1)];
    hcoup = r * Ts[mm * ldT + mm] / tmm;
    for (int i = tid; i < mm; i += kThreads) Xs[i * kMaxM + (mm - 1)] += (r / tmm) * Ts[i * ldT + mm];
  }
  const double beta = st->alpha * Ts[0];
  __syncthreads();
  for (int e = tid; e < m * m; e += kThreads) {
    const int i = e % m, c = e / m;
    a.Xout[e] = (i < mm && c < mm) ? Xs[i * kMaxM + c] : 0.0;
  }
  if (tid == 0) {
    st->beta = beta;
    st->h = hcoup;
  }

  // ---- 3. quadrature solves (zeta_l I - X) y = e_1, one system per thread
  const int nq_tot = a.nq_main + a.nq_chk;
  const int nsys = nt * nq_tot;
  for (int s = tid; s < nsys; s += kThreads) hess_solve(mm, Xs, kMaxM, a.rz[s], a.scr + s, a.ldscr);
  __syncthreads();

  // ---- 4. g_t = beta * sum_l w_l psi_l y_l  (twice the real part for conjugate-half rules)
  const double fac = (a.fun == 0) ? 2.0 : 1.0;
  for (int e = tid; e < 2 * nt * mm; e += kThreads) {
    const int rule = e / (nt * mm), rem = e % (nt * mm), it = rem / mm, i = rem % mm;
    const int l0 = it * nq_tot + (rule ? a.nq_main : 0);
    const int l1 = l0 + (rule ? a.nq_chk : a.nq_main);
    double acc = 0.0;
    for (int l = l0; l < l1; ++l) {
      const cplx y = a.scr[(size_t)i * a.ldscr + l];
      const cplx wp = cmul(a.rw[l], a.psi[l]);
      acc += wp.re * y.re - wp.im * y.im;
    }
    a.gbuf[(size_t)rule * nt * m + (size_t)it * m + i] = fac * beta * acc;
  }
  __syncthreads();
  // psi_l <- psi_l * beta * h * [y_l]_m
  for (int s = tid; s < nsys; s += kThreads) {
    const cplx ym = a.scr[(size_t)(mm - 1) * a.ldscr + s];
    a.psi[s] = cscale(cmul(a.psi[s], ym), beta * hcoup);
  }

  // ---- 5. pass coefficients: C[:, t] = T_m^{-1} g_t ; C[:, nt] = restart vector coefficients
  for (int it = tid; it <= nt; it += kThreads) {
    double* col = a.C + (size_t)it * C_ld;
    if (it < nt) {
      const double* g = a.gbuf + (size_t)it * m;
      for (int i = mm - 1; i >= 0; --i) {
        double s = g[i];
        for (int l = i + 1; l < mm; ++l) s -= Ts[i * ldT + l] * col[l];
        col[i] = s / Ts[i * ldT + i];
      }
      // disagreement of the two rules, measured in the sketch-orthonormal coordinates
      const double* gc = a.gbuf + (size_t)nt * m + (size_t)it * m;
      double q2 = 0.0;
      for (int i = 0; i < mm; ++i) q2 += (g[i] - gc[i]) * (g[i] - gc[i]);
      st->qdis2[it] = q2;
    } else if (!brk) {
      // v_hat = (w_{m+1} - W_m T_m^{-1} t) / tau
      const double tau = Ts[mm * ldT + mm];
      for (int i = mm - 1; i >= 0; --i) {
        double s = Ts[i * ldT + mm];
        for (int l = i + 1; l < mm; ++l) s -= Ts[i * ldT + l] * (-col[l] * tau);
        col[i] = -(s / Ts[i * ldT + i]) / tau;
      }
      col[mm] = 1.0 / tau;
    }
  }
}

// ------------------------------------------------------------------------------ fused pass
// x_t += W c_t for every time point, v_hat = W c_nt written over column 0, and per-block
// partial norms ||y_t||^2, ||x_t||^2 (added into kSlots copies).
template <typename T, int NT>
__global__ __launch_bounds__(kThreads) void k_pass(int n, int m, int nt, const double* __restrict__ C,
                                                   T* __restrict__ W, double* __restrict__ x,
                                                   double* __restrict__ norm_slots, const State* __restrict__ st) {
  __shared__ double Cs[(kMaxM + 1) * (NT + 1)];
  __shared__ double part[kThreads / 64][2 * NT];
  const int mm = st->meff;
  if (st->nonfinite || mm == 0) return;
  const int brk = st->brk;
  const int ncol = brk ? mm : mm + 1;
  for (int e = threadIdx.x; e < (m + 1) * (nt + 1); e += kThreads) {
    const int i = e % (m + 1), c = e / (m + 1);
    Cs[i * (NT + 1) + (c < nt ? c : NT)] = C[e];
  }
  __syncthreads();
  double yn[NT], xn[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) yn[q] = xn[q] = 0.0;
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < (size_t)n; i += stride) {
    double acc[NT + 1];
#pragma unroll
    for (int q = 0; q <= NT; ++q) acc[q] = 0.0;
    for (int j = 0; j < ncol; ++j) {
      const double w = (double)W[(size_t)j * n + i];
#pragma unroll
      for (int q = 0; q <= NT; ++q) acc[q] = fma(w, Cs[j * (NT + 1) + q], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (q < nt) {
        double* xp = x + (size_t)q * n + i;
        const double xv = *xp + acc[q];
        *xp = xv;
        yn[q] += acc[q] * acc[q];
        xn[q] += xv * xv;
      }
    }
    if (!brk) W[i] = (T)acc[NT];
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
  if (threadIdx.x < 2 * nt) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += part[q][threadIdx.x];
    unsafeAtomicAdd(norm_slots + (size_t)(blockIdx.x % kSlots) * (2 * kMaxNt) + threadIdx.x, s);
  }
}

// Convergence test after the pass (Algorithm 2 stopping rule, relative form).
__global__ void k_final(int nt, double tol, double* __restrict__ norm_slots, State* __restrict__ st,
                        Report* __restrict__ rep) {
  if (threadIdx.x != 0) return;
  double est = 0.0, qd = 0.0;
  for (int it = 0; it < nt; ++it) {
    double y2 = 0.0, x2 = 0.0;
    for (int q = 0; q < kSlots; ++q) {
      y2 += norm_slots[(size_t)q * (2 * kMaxNt) + 2 * it];
      x2 += norm_slots[(size_t)q * (2 * kMaxNt) + 2 * it + 1];
    }
    st->ynorm2[it] = y2;
    st->xnorm2[it] = x2;
    const double e = (x2 > 0.0) ? sqrt(y2 / x2) : 0.0;
    const double qq = (x2 > 0.0) ? sqrt(st->qdis2[it] / x2) : 0.0;
    est = fmax(est, e);
    qd = fmax(qd, qq);
  }
  for (int q = 0; q < kSlots * 2 * kMaxNt; ++q) norm_slots[q] = 0.0;
  st->est = est;
  st->qdis_rel = qd;
  st->converged = (est <= tol) ? 1 : 0;
  rep->est = est;
  rep->qdis_rel = qd;
  rep->alpha = st->alpha;
  rep->beta = st->beta;
  rep->brk = st->brk;
  rep->meff = st->meff;
  rep->nonfinite = st->nonfinite;
  rep->converged = st->converged;
}

// Sum of the slot copies: out[i] = sum_c slots[c*len + i] (sketch test hook).
__global__ void k_reduce_slots(int len, const double* __restrict__ slots, double* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < kSlots; ++c) s += slots[(size_t)c * len + i];
    out[i] = s;
  }
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

// ------------------------------------------------------------------------------------ launchers
hipError_t launch_zero(hipStream_t s, double* p, size_t count) {
  if (count == 0) return hipSuccess;
  int grid = (int)((count + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_rule(hipStream_t s, int fun, int nt, const double* tvals, int n_main, double lo, double hi,
                       cplx* rz, cplx* rw, cplx* psi) {
  hipLaunchKernelGGL(k_rule, dim3(8), dim3(256), 0, s, fun, nt, tvals, n_main, lo, hi, rz, rw, psi);
  return hipGetLastError();
}

hipError_t launch_copy_in(hipStream_t s, int dtype, int grid, int n, const void* b, void* w0) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_copy_in<double>, dim3(grid), dim3(256), 0, s, n, (const double*)b, (double*)w0);
  else
    hipLaunchKernelGGL(k_copy_in<float>, dim3(grid), dim3(256), 0, s, n, (const float*)b, (float*)w0);
  return hipGetLastError();
}

hipError_t launch_sqnorm(hipStream_t s, int dtype, int grid, int n, const void* v, double* slots) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_sqnorm<double>, dim3(grid), dim3(kThreads), 0, s, n, (const double*)v, slots);
  else
    hipLaunchKernelGGL(k_sqnorm<float>, dim3(grid), dim3(kThreads), 0, s, n, (const float*)v, slots);
  return hipGetLastError();
}

hipError_t launch_start(hipStream_t s, int d, int m, int plain, double* slots_start, double* slots_step,
                        size_t step_len, double* U, double* R, State* st) {
  hipLaunchKernelGGL(k_start, dim3(1), dim3(kThreads), 0, s, d, m, plain, slots_start, slots_step, step_len, U, R,
                     st);
  return hipGetLastError();
}

hipError_t launch_small(hipStream_t s, const SmallArgs& a) {
  hipLaunchKernelGGL(k_small, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T>
static void launch_pass_t(hipStream_t s, int grid, int n, int m, int nt, const double* C, T* W, double* x,
                          double* ns, const State* st) {
  if (nt <= 1)
    hipLaunchKernelGGL((k_pass<T, 1>), dim3(grid), dim3(kThreads), 0, s, n, m, nt, C, W, x, ns, st);
  else if (nt <= 2)
    hipLaunchKernelGGL((k_pass<T, 2>), dim3(grid), dim3(kThreads), 0, s, n, m, nt, C, W, x, ns, st);
  else if (nt <= 4)
    hipLaunchKernelGGL((k_pass<T, 4>), dim3(grid), dim3(kThreads), 0, s, n, m, nt, C, W, x, ns, st);
  else if (nt <= 8)
    hipLaunchKernelGGL((k_pass<T, 8>), dim3(grid), dim3(kThreads), 0, s, n, m, nt, C, W, x, ns, st);
  else
    hipLaunchKernelGGL((k_pass<T, 16>), dim3(grid), dim3(kThreads), 0, s, n, m, nt, C, W, x, ns, st);
}

hipError_t launch_pass(hipStream_t s, int dtype, int grid, int n, int m, int nt, const double* C, void* W,
                       double* x, double* norm_slots, const State* st) {
  if (dtype == 0)
    launch_pass_t<double>(s, grid, n, m, nt, C, (double*)W, x, norm_slots, st);
  else
    launch_pass_t<float>(s, grid, n, m, nt, C, (float*)W, x, norm_slots, st);
  return hipGetLastError();
}

hipError_t launch_final(hipStream_t s, int nt, double tol, double* norm_slots, State* st, Report* rep) {
  hipLaunchKernelGGL(k_final, dim3(1), dim3(64), 0, s, nt, tol, norm_slots, st, rep);
  return hipGetLastError();
}

hipError_t launch_reduce_slots(hipStream_t s, int len, const double* slots, double* out) {
  hipLaunchKernelGGL(k_reduce_slots, dim3((len + 255) / 256), dim3(256), 0, s, len, slots, out);
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

}  // namespace fab
