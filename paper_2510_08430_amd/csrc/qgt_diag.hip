// Diagnostics of the inverse block-layer QGT against a reference inverse
// (paper, Sec. 3, Eq. 4 (a) Frobenius overlap and (b) Frobenius relative
// error), computed on the device from the Cholesky factors a solve leaves in
// the workspace.
//
// For a problem whose blocks are all in parameter form, the inverse of the
// shifted block-layer QGT is A = diag(A_1, ..., A_L), A_b = (L_b L_b^H)^{-1}
// = X_b^H X_b with X_b = L_b^{-1}.  Given a reference B (n_p x n_p, complex
// FP64), the kernels form
//   s[0] = Re sum_b sum_ij conj(A_b)_ij B_(b)ij      (Re Tr[A^H B], A block-diagonal)
//   s[1] = sum_b ||A_b||_F^2
//   s[2] = ||B||_F^2
//   s[3] = sum_b ||A_b - B_bb||_F^2
//   s[4] = sum_b ||B_bb||_F^2
// so that F(A, B) = s0 / sqrt(s1 s2) and eps_F(A, B) = sqrt(s3 + s2 - s4) /
// sqrt(s2).  All sums are FP64 in a fixed order (per-workgroup partials, then
// one ordered reduction), so repeated calls give identical results.
#include <vector>

#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

// X = L^{-1} of one block by forward substitution, one workgroup per column j:
// x_i = (delta_ij - sum_{j<=k<i} L_ik x_k) / L_ii for i = j .. m-1 (x_i = 0
// above the diagonal).  The column is kept in LDS; each step reduces over the
// workgroup.  X is m x m row-major (leading dimension ldx) in the scratch.
template <typename T>
__device__ void trtri_column(const T* L, int64_t ld, int m, int j, double2* X, int64_t ldx, double2* xs,
                             double2* red) {
  const int t = threadIdx.x;
  for (int i = t; i < m; i += 256) xs[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = j; i < m; ++i) {
    double2 acc = make_double2(0.0, 0.0);
    const T* Li = L + (int64_t)i * ld * 2;
    for (int k = j + t; k < i; k += 256) {
      const double2 l = make_double2((double)Li[2 * k], (double)Li[2 * k + 1]);
      acc = cfma(l, xs[k], acc);
    }
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      double2 s = make_double2(i == j ? 1.0 : 0.0, 0.0);
      for (int w = 0; w < 4; ++w) s = csub(s, red[w]);
      const double lii = (double)Li[2 * i];  // the diagonal of L is real and positive
      xs[i] = cscale(s, 1.0 / lii);
    }
    __syncthreads();
  }
  for (int i = t; i < m; i += 256) X[(int64_t)i * ldx + j] = xs[i];
}

__global__ void __launch_bounds__(256) k_trtri_cols(const BlockDev* blocks, int g, const char* ws, double2* X,
                                                    int64_t ldx) {
  extern __shared__ double2 xs[];
  __shared__ double2 red[4];
  const BlockDev B = blocks[g];
  const int j = blockIdx.x;
  if (j >= B.m) return;
  if (B.fact32) trtri_column<float>(ws_at<float>(ws, B.mat_off), B.m_pad, (int)B.m, j, X, ldx, xs, red);
  else trtri_column<double>(ws_at<double>(ws, B.mat_off), B.m_pad, (int)B.m, j, X, ldx, xs, red);
}

// Partial sums of one row of entries (i, 0..m-1) of A_b = X^H X against the
// reference: A_ij = sum_{k >= max(i,j)} conj(X_ki) X_kj.  One workgroup per
// row i; part[5 * (row_base + i) + q] receives the row's five sums.
__global__ void __launch_bounds__(256) k_inverse_sums(const BlockDev* blocks, int g, const double2* X, int64_t ldx,
                                                      const double2* Bref, int64_t ldb, double* part,
                                                      int row_base) {
  const BlockDev Bk = blocks[g];
  const int m = (int)Bk.m, i = blockIdx.x, t = threadIdx.x;
  if (i >= m) return;
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = t; j < m; j += 256) {
    double2 a = make_double2(0.0, 0.0);
    for (int k = i > j ? i : j; k < m; ++k) a = cfma(cconj(X[(int64_t)k * ldx + i]), X[(int64_t)k * ldx + j], a);
    const double2 b = Bref[(Bk.col_off + i) * ldb + Bk.col_off + j];
    s[0] += a.x * b.x + a.y * b.y;
    s[1] += a.x * a.x + a.y * a.y;
    s[3] += (a.x - b.x) * (a.x - b.x) + (a.y - b.y) * (a.y - b.y);
    s[4] += b.x * b.x + b.y * b.y;
  }
  __shared__ double red[4][5];
  for (int q = 0; q < 5; ++q) {
    const double v = wave_sum(s[q]);
    if ((t & 63) == 0) red[t >> 6][q] = v;
  }
  __syncthreads();
  if (t < 5) part[(int64_t)5 * (row_base + i) + t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
}

// ||B||_F^2 by rows: part2[r] for row r of the reference (n_p rows).
__global__ void __launch_bounds__(256) k_ref_norm(const double2* Bref, int64_t ldb, int64_t n, double* part2) {
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < n; c += 256) {
    const double2 b = Bref[r * ldb + c];
    s += b.x * b.x + b.y * b.y;
  }
  __shared__ double red[4];
  const double v = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part2[r] = red[0] + red[1] + red[2] + red[3];
}

// Ordered final sums: out[q] = sum over rows of part (q != 2) or part2 (q = 2).
__global__ void __launch_bounds__(64) k_diag_final(const double* part, int nrows, const double* part2, int64_t n,
                                                   double* out) {
  const int q = threadIdx.x;
  if (q >= 5) return;
  double s = 0.0;
  if (q == 2)
    for (int64_t r = 0; r < n; ++r) s += part2[r];
  else
    for (int r = 0; r < nrows; ++r) s += part[(int64_t)5 * r + q];
  out[q] = s;
}

void launch_block_inverse_sums(const BlockDev* blocks, const std::vector<int>& glist, const std::vector<int64_t>& m,
                               const char* ws, double2* X, int64_t ldx, const double2* Bref, int64_t ldb, int64_t n_p,
                               double* part, double* part2, double* out, hipStream_t s) {
  int row_base = 0;
  for (size_t x = 0; x < glist.size(); ++x) {
    const int g = glist[x];
    const unsigned mm = (unsigned)m[x];
    hipLaunchKernelGGL(k_trtri_cols, dim3(mm), dim3(256), (size_t)mm * sizeof(double2), s, blocks, g, ws, X, ldx);
    hipLaunchKernelGGL(k_inverse_sums, dim3(mm), dim3(256), 0, s, blocks, g, X, ldx, Bref, ldb, part, row_base);
    row_base += (int)mm;
  }
  hipLaunchKernelGGL(k_ref_norm, dim3((unsigned)n_p), dim3(256), 0, s, Bref, ldb, n_p, part2);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, part, row_base, part2, n_p, out);
}

}  // namespace qgt
