// Host-core comparator: plain restarted Arnoldi for exp(-tA) b on CPU threads (FP64, OpenMP).
//
// The method the sketched solver is measured against, run on the host instead of the GPU: each
// cycle builds an orthonormal Krylov basis by classical Gram-Schmidt applied twice (the Arnoldi
// process of the paper's Section 2 with a stable orthogonalisation), and the restart is the same
// quadrature recursion the GPU library uses (Section 4): for the nodes zeta_l and weights w_l of a
// rule for exp(-t z),
//   c = alpha * sum_l fac * Re(w_l psi_l (zeta_l - H_m)^{-1} e_1),   x += V_m c,
//   psi_l <- psi_l * alpha * h_{m+1,m} * e_m^T (zeta_l - H_m)^{-1} e_1,
// with the next cycle starting from v_{m+1}.  The rule is the parabolic Hankel contour
// s(u) = P - mu u^2 + 2 i mu u in s = -t z, midpoint rule with N nodes, of which the N/2 with
// Im s < 0 are solved and the result doubled in its real part (conjugate symmetry).  The stopping
// test is the library's: the successive difference ||V_m c|| / ||x|| continued by the geometric
// tail q / (1 - q) of the increments' contraction ratio q (the largest of the last three), or the
// difference alone once it is at the FP64 unit roundoff, stopping when that is <= tol.
//
// It is neither the oracle nor the product: it shares no code with either and exists to time the
// plain method on the host cores of the GPU machine.
#include <omp.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <vector>

namespace {

using cd = std::complex<double>;

constexpr double kP = 3.0, kMu = 6.0, kL = 45.0;  // contour parameters (shared with the GPU rule)

void spmv(int64_t n, const int32_t* rp, const int32_t* ci, const double* va, const double* x, double* y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s += va[p] * x[ci[p]];
    y[i] = s;
  }
}

// h[0..nc) = V[:, 0..nc)^T z, V column-major with leading dimension n.
void gram(int64_t n, int nc, const double* V, const double* z, double* h) {
  const int nth = omp_get_max_threads();
  std::vector<double> part((size_t)nth * nc, 0.0);
#pragma omp parallel
  {
    std::vector<double> loc(nc, 0.0);  // private accumulators, copied out once
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const double zi = z[i];
      for (int c = 0; c < nc; ++c) loc[c] += V[(size_t)c * n + i] * zi;
    }
    std::copy(loc.begin(), loc.end(), part.begin() + (size_t)omp_get_thread_num() * nc);
  }
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int q = 0; q < nth; ++q) s += part[(size_t)q * nc + c];
    h[c] = s;
  }
}

// z -= V[:, 0..nc) h; returns ||z||^2 after the update.
double subtract(int64_t n, int nc, const double* V, const double* h, double* z) {
  double nrm = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : nrm)
  for (int64_t i = 0; i < n; ++i) {
    double v = z[i];
    for (int c = 0; c < nc; ++c) v -= V[(size_t)c * n + i] * h[c];
    z[i] = v;
    nrm += v * v;
  }
  return nrm;
}

// y = (zeta - H)^{-1} e_1 for the m x m upper Hessenberg H (column-major, leading dimension ldh),
// by Gaussian elimination with partial pivoting between neighbouring rows.
void hess_solve(int m, const double* H, int ldh, cd zeta, cd* y, std::vector<cd>& M) {
  M.assign((size_t)m * m, cd(0.0));
  for (int c = 0; c < m; ++c)
    for (int r = 0; r <= std::min(c + 1, m - 1); ++r) M[(size_t)c * m + r] = (r == c ? zeta : cd(0.0)) - H[(size_t)c * ldh + r];
  std::vector<cd> rhs(m, cd(0.0));
  rhs[0] = 1.0;
  for (int r = 0; r < m - 1; ++r) {
    if (std::abs(M[(size_t)r * m + r + 1]) > std::abs(M[(size_t)r * m + r])) {  // swap rows r, r+1
      for (int c = r; c < m; ++c) std::swap(M[(size_t)c * m + r], M[(size_t)c * m + r + 1]);
      std::swap(rhs[r], rhs[r + 1]);
    }
    const cd piv = M[(size_t)r * m + r];
    const cd f = (piv == cd(0.0)) ? cd(0.0) : M[(size_t)r * m + r + 1] / piv;
    for (int c = r; c < m; ++c) M[(size_t)c * m + r + 1] -= f * M[(size_t)c * m + r];
    rhs[r + 1] -= f * rhs[r];
  }
  for (int r = m - 1; r >= 0; --r) {
    cd s = rhs[r];
    for (int c = r + 1; c < m; ++c) s -= M[(size_t)c * m + r] * y[c];
    y[r] = s / M[(size_t)r * m + r];
  }
}

}  // namespace

extern "C" {

// OpenMP threads a call uses (OMP_NUM_THREADS, else the host's count).
int cpu_plain_threads(void) { return omp_get_max_threads(); }

// x (n, FP64, overwritten) <- approximation of exp(-tA) b.  Returns 0 when the stopping test was
// met, 1 on a breakdown (exact result), 2 when max_cycles ran out, -1 on invalid arguments.
// *cycles and *matvecs receive the work done.  n_quad: nodes of the contour rule (even, 0 = 128).
int cpu_plain_expv(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* vals, const double* b,
                   double t, int m, double tol, int max_cycles, int n_quad, double* x, int* cycles,
                   int* matvecs) {
  if (n < 1 || m < 1 || !(t > 0.0) || max_cycles < 1 || !rowptr || !colind || !vals || !b || !x) return -1;
  const int N = n_quad > 0 ? n_quad : 128;
  if (N % 2) return -1;
  const int nq = N / 2;
  std::vector<cd> zeta(nq), w(nq), psi(nq, cd(1.0));
  {
    const double U = std::sqrt((kP + kL) / kMu), h = 2.0 * U / N;
    for (int l = 0; l < nq; ++l) {
      const double u = -U + (l + 0.5) * h;
      const cd s(kP - kMu * u * u, 2.0 * kMu * u), ds(-2.0 * kMu * u, 2.0 * kMu);
      zeta[l] = -s / t;
      w[l] = (h / (2.0 * M_PI * t)) * cd(0.0, 1.0) * ds * std::exp(s);
    }
  }
  std::vector<double> V((size_t)n * (m + 1)), H((size_t)(m + 1) * m), hv(m + 1), hv2(m + 1), c(m);
  std::vector<cd> y(m), M;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    x[i] = 0.0;
    V[i] = b[i];
  }
  int status = 2, cyc = 0, mv = 0;
  double yprev = 0.0, qprev = 0.0, qprev2 = 0.0;  // the stopping test's last increment norm and ratios
  for (cyc = 1; cyc <= max_cycles; ++cyc) {
    double a2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : a2)
    for (int64_t i = 0; i < n; ++i) a2 += V[i] * V[i];
    const double alpha = std::sqrt(a2);
    if (!(alpha > 0.0)) {
      status = 1;
      break;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) V[i] /= alpha;
    std::fill(H.begin(), H.end(), 0.0);
    int mm = m;
    bool brk = false;
    for (int j = 0; j < m; ++j) {
      double* z = V.data() + (size_t)(j + 1) * n;
      spmv(n, rowptr, colind, vals, V.data() + (size_t)j * n, z);
      ++mv;
      double raw2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : raw2)
      for (int64_t i = 0; i < n; ++i) raw2 += z[i] * z[i];
      gram(n, j + 1, V.data(), z, hv.data());
      subtract(n, j + 1, V.data(), hv.data(), z);
      gram(n, j + 1, V.data(), z, hv2.data());
      const double r2 = subtract(n, j + 1, V.data(), hv2.data(), z);
      for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] = hv[i] + hv2[i];
      const double rho = std::sqrt(r2);
      if (!(rho > 64.0 * 2.220446049250313e-16 * std::sqrt(raw2))) {  // invariant subspace: exact
        mm = j + 1;
        brk = true;
        break;
      }
      H[(size_t)j * (m + 1) + j + 1] = rho;
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) z[i] /= rho;
    }
    const double hnext = brk ? 0.0 : H[(size_t)(mm - 1) * (m + 1) + mm];
    std::fill(c.begin(), c.end(), 0.0);
    for (int l = 0; l < nq; ++l) {
      hess_solve(mm, H.data(), m + 1, zeta[l], y.data(), M);
      const cd wp = w[l] * psi[l];
      for (int i = 0; i < mm; ++i) c[i] += 2.0 * alpha * (wp * y[i]).real();
      psi[l] *= y[mm - 1] * (alpha * hnext);
    }
    double y2 = 0.0, x2 = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : y2, x2)
    for (int64_t i = 0; i < n; ++i) {
      double u = 0.0;
      for (int k = 0; k < mm; ++k) u += V[(size_t)k * n + i] * c[k];
      x[i] += u;
      y2 += u * u;
      x2 += x[i] * x[i];
    }
    if (brk) {
      status = 1;
      break;
    }
    {  // remaining-error estimate: the geometric tail of the increments (the library's stopping test)
      const double yn = std::sqrt(y2), rel = x2 > 0.0 ? std::sqrt(y2 / x2) : 0.0;
      const double inf = std::numeric_limits<double>::infinity();
      const double q = (cyc == 1) ? inf : (yprev > 0.0 ? yn / yprev : (yn > 0.0 ? inf : 0.0));
      double qb = q;  // the largest of the last three ratios
      if (cyc >= 3) qb = std::max(qb, qprev);
      if (cyc >= 4) qb = std::max(qb, qprev2);
      const double est = (rel <= 0x1p-53) ? rel : (qb < 1.0 ? rel * qb / (1.0 - qb) : inf);  // roundoff: noise
      yprev = yn;
      qprev2 = qprev;
      qprev = q;
      if (est <= tol) {
        status = 0;
        break;
      }
    }
    if (cyc == max_cycles) break;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) V[i] = V[(size_t)m * n + i];  // next start vector v_{m+1}
  }
  if (cycles) *cycles = std::min(cyc, max_cycles);
  if (matvecs) *matvecs = mv;
  return status;
}

}  // extern "C"
