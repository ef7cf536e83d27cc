// Information metrics s(F) of eq:cost_info (trace, smallest eigenvalue,
// log-determinant) on a symmetric 6x6 FIM held as 21 FP64 values, and their
// gradients dS/dF for the backward pass.
#pragma once

#include "fif_device.h"

namespace fif {

constexpr uint32_t M_TRACE = 1u, M_LMIN = 2u, M_LOGDET = 4u, M_FIM = 8u;
constexpr uint8_t FL_CLAMPED = 1u, FL_NOT_PD = 2u, FL_TIE = 4u;

// Writes the requested columns to `row` (when non-null), sets flag bits, and
// when GRAD accumulates G = sum_c up[c] d s_c / dF (21, symmetric).
template <bool GRAD>
__device__ inline void eval_metrics(const double F[21], uint32_t metrics, double* row,
                                    uint8_t* flag, const double* up, double G[21],
                                    bool want_pd = true) {
  int col = 0, upc = 0;
  // up[upc] with constant indices only (a runtime index would put up in scratch)
  auto upat = [&](int c) { return c == 0 ? up[0] : (c == 1 ? up[1] : up[2]); };
  if (GRAD) {
#pragma unroll
    for (int e = 0; e < 21; ++e) G[e] = 0.0;
  }
  if (metrics & M_TRACE) {
    double tr = F[u21(0, 0)] + F[u21(1, 1)] + F[u21(2, 2)] + F[u21(3, 3)] + F[u21(4, 4)] +
                F[u21(5, 5)];
    if (row) row[col] = tr;
    ++col;
    if (GRAD) {
      double g = upat(upc++);
#pragma unroll
      for (int i = 0; i < 6; ++i) G[u21(i, i)] += g;
    }
  }
  if (metrics & M_LMIN) {
    double a[21];
#pragma unroll
    for (int e = 0; e < 21; ++e) a[e] = F[e];
    jacobi6<false>(a, nullptr);
    double ev[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ev[i] = a[u21(i, i)];
    double lmin = ev[0], amax = fabs(ev[0]);
    int imin = 0;
#pragma unroll
    for (int i = 1; i < 6; ++i) {
      bool lt = ev[i] < lmin;
      lmin = lt ? ev[i] : lmin;
      imin = lt ? i : imin;
      amax = fmax(amax, fabs(ev[i]));
    }
    double second = __builtin_inf();
#pragma unroll
    for (int i = 0; i < 6; ++i) second = (i != imin) ? fmin(second, ev[i]) : second;
    if (second - lmin <= 1e-8 * amax) *flag |= FL_TIE;
    if (row) row[col] = lmin;
    ++col;
    if (GRAD) {
      // d lambda_min / dF = v v^T with v the unit eigenvector (undefined at a
      // tie, which is flagged); v by inverse iteration with the shift
      // 1e-10 max|lambda| below lambda_min, more than the Jacobi error of
      // lambda_min (1e-11 |F|), so that F - sigma I stays positive definite
      double g = upat(upc++);
      double v[6];
      lmin_vector6(F, lmin - fmax(1e-10 * amax, 1e-300), v);
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) G[u21(i, j)] = fma(g * v[i], v[j], G[u21(i, j)]);
    }
  }
  if (want_pd || (metrics & M_LOGDET)) {
    double L[36], dinv[6], ld;
    bool pd = ldlt6(F, L, dinv, &ld);
    if (!pd) *flag |= FL_NOT_PD;
    if (metrics & M_LOGDET) {
      if (row) row[col] = ld;
      ++col;
      if (GRAD) {
        double g = upat(upc++);
        double inv[21];
        ldlt6_inverse(L, dinv, inv);
        // a zero weight leaves the log-det out of L, so a FIM that is not
        // positive definite does not turn the other metrics' gradient to NaN
#pragma unroll
        for (int e = 0; e < 21; ++e)
          G[e] = (g == 0.0) ? G[e] : (pd ? fma(g, inv[e], G[e]) : __builtin_nan(""));
      }
    }
  }
  if ((metrics & M_FIM) && row) {
#pragma unroll
    for (int e = 0; e < 21; ++e) row[col + e] = F[e];
  }
}

}  // namespace fif
