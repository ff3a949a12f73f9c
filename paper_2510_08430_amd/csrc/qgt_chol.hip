// FP64 blocked Cholesky factorisation and triangular solves for the shifted
// block matrices (S_b + lambda I or the sample-space T_b + lambda I), batched
// over all blocks of all problems.  The matrices are Hermitian positive
// definite because lambda > 0, so the factorisation needs no pivoting.
//
// Storage: row-major m_pad x m_pad complex128, lower triangle, 64x64 tiles.
// Right-looking tile algorithm, step k:
//   POTRF  : L_kk L_kk^H = A_kk (one workgroup, in LDS) and Linv_kk = L_kk^{-1}
//   TRSM   : L_ik = A_ik Linv_kk^H                           (i > k)
//   UPDATE : A_ij -= L_ik L_jk^H                              (i >= j > k)
// TRSM and UPDATE are the same tile product C = beta C + alpha X Y^H on the
// FP64 matrix cores (v_mfma_f64_16x16x4_f64, four real products per complex
// product).  Triangular solves use the stored Linv_kk for the diagonal tiles.
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

// ---------------------------------------------------------------------------
// POTRF of diagonal tile k of every listed block, plus the inverse of the
// factor.  Non-positive or non-finite pivots are recorded in status[g] and
// replaced by 1 so that the factorisation still terminates.
__global__ void __launch_bounds__(256) k_potrf(const int32_t* glist, const BlockDev* blocks, char* ws, int k,
                                               int32_t* status) {
  __shared__ double2 L[64][65];
  __shared__ double2 X[64][65];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int g = glist[blockIdx.x];
  const BlockDev B = blocks[g];
  if (k >= B.ntiles) return;
  double2* A = ws_at<double2>(ws, B.mat_off) + ((int64_t)k * 64) * B.m_pad + (int64_t)k * 64;
  if (t == 0) bad = 0;
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    L[i][j] = j <= i ? A[(int64_t)i * B.m_pad + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    double d = L[j][j].x;
    const bool ok = d > 0.0 && d < INFINITY;
    if (!ok) d = 1.0;
    const double ljj = sqrt(d), inv = 1.0 / ljj;
    __syncthreads();
    if (t == 0) {
      L[j][j] = make_double2(ljj, 0.0);
      if (!ok) bad = 1;
    }
    if (t > j && t < 64) L[t][j] = cscale(L[t][j], inv);
    __syncthreads();
    const int n = 63 - j;
    for (int idx = t; idx < n * n; idx += 256) {
      const int i = j + 1 + idx / n, c = j + 1 + idx % n;
      if (c <= i) {
        const double2 a = L[i][j], b = L[c][j];
        // L[i][c] -= a * conj(b)
        L[i][c] = make_double2(L[i][c].x - (a.x * b.x + a.y * b.y), L[i][c].y - (a.y * b.x - a.x * b.y));
      }
    }
    __syncthreads();
  }
  // X = L^{-1}: row sweep, column c of X in thread c (entries i >= c).
  for (int i = 0; i < 64; ++i) {
    if (t <= i) {
      const int c = t;
      double2 s = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int q = c; q < i; ++q) {
        const double2 a = L[i][q], x = X[q][c];
        s = make_double2(s.x - (a.x * x.x - a.y * x.y), s.y - (a.x * x.y + a.y * x.x));
      }
      const double inv = 1.0 / L[i][i].x;
      X[i][c] = cscale(s, inv);
    }
    __syncthreads();
  }
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    if (j <= i) A[(int64_t)i * B.m_pad + j] = L[i][j];
  }
  double2* Li = ws_at<double2>(ws, B.linv_off) + (int64_t)k * 4096;
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    Li[idx] = j <= i ? X[i][j] : make_double2(0.0, 0.0);
  }
  if (t == 0 && bad) status[g] = 5;  // QGT_ERR_NOT_POSITIVE_DEFINITE
}

// ---------------------------------------------------------------------------
// Tile product C = X Y^H (TRSM: X = A_ik, Y = Linv_kk, C = A_ik in place) or
// C -= X Y^H (UPDATE: X = L_ik, Y = L_jk, C = A_ij).  64x64 output, K = 64 in
// four LDS stages of 16.  Complex product with real MFMAs:
//   X = a + ib, Y = c + id:  Re(X Y^H) = a c^T + b d^T,  Im(X Y^H) = b c^T - a d^T.
template <int MODE>  // 0 = TRSM, 1 = UPDATE
__global__ void __launch_bounds__(256) k_tile_gemm(const TileTask* tasks, const BlockDev* blocks, char* ws, int k) {
  __shared__ double2 Xs[64][17];
  __shared__ double2 Ys[64][17];
  const TileTask tk = tasks[blockIdx.x];
  const BlockDev B = blocks[tk.g];
  const int64_t ld = B.m_pad;
  double2* Abase = ws_at<double2>(ws, B.mat_off);
  double2* Cp = Abase + ((int64_t)tk.i * 64) * ld + (int64_t)tk.j * 64;
  const double2* Xp;
  const double2* Yp;
  int64_t ldy;
  if (MODE == 0) {
    Xp = Abase + ((int64_t)tk.i * 64) * ld + (int64_t)k * 64;
    Yp = ws_at<double2>(ws, B.linv_off) + (int64_t)k * 4096;
    ldy = 64;
  } else {
    Xp = Abase + ((int64_t)tk.i * 64) * ld + (int64_t)k * 64;
    Yp = Abase + ((int64_t)tk.j * 64) * ld + (int64_t)k * 64;
    ldy = ld;
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1, l16 = lane & 15, lg = lane >> 4;
  d4v accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }

  const int lrow = t >> 2, lq = t & 3;  // loader: row, quarter of 16 columns
  for (int st = 0; st < 4; ++st) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Xs[lrow][lq * 4 + e] = Xp[(int64_t)lrow * ld + st * 16 + lq * 4 + e];
      Ys[lrow][lq * 4 + e] = Yp[(int64_t)lrow * ldy + st * 16 + lq * 4 + e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = 4 * lg + e;
      double2 xa[2], yb[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        xa[s] = Xs[32 * wr + 16 * s + l16][kk];
        yb[s] = Ys[32 * wc + 16 * s + l16][kk];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].x, yb[b].x, accR[a][b], 0, 0, 0);
          accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].y, yb[b].y, accR[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a].y, yb[b].x, accI[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xa[a].x, yb[b].y, accI[a][b], 0, 0, 0);
        }
    }
  }
  __syncthreads();  // TRSM writes C = X in place: all reads of X are done
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int iloc = 32 * wr + 16 * a + 4 * r + lg;
        const int jloc = 32 * wc + 16 * b + l16;
        double2* c = Cp + (int64_t)iloc * ld + jloc;
        if (MODE == 0) {
          *c = make_double2(accR[a][b][r], accI[a][b][r]);
        } else {
          const double2 old = *c;
          *c = make_double2(old.x - accR[a][b][r], old.y - accI[a][b][r]);
        }
      }
}

// ---------------------------------------------------------------------------
// Triangular solves, one launch per tile step, all listed blocks at once.
// Forward (L y = r), step k, workgroup (i, g) with i >= k:
//   y_k = Linv_kk r_k; the workgroup i == k stores y_k, the others update
//   r_i -= L_ik y_k.
// Backward (L^H c = y), step k descending, workgroup (i, g) with i <= k:
//   c_k = Linv_kk^H y_k; i == k adds c_k to the solution x, the others update
//   y_i -= L_ki^H c_k.
// 256 threads: 4 threads per row (or column) of the 64x64 tile, each summing 16
// products, combined with lane shuffles.
__device__ __forceinline__ double2 quad_sum(double2 v) {
  v.x += __shfl_xor(v.x, 1, 64);
  v.y += __shfl_xor(v.y, 1, 64);
  v.x += __shfl_xor(v.x, 2, 64);
  v.y += __shfl_xor(v.y, 2, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_trsv_fwd(const int32_t* glist, const BlockDev* blocks, char* ws, int k) {
  __shared__ double2 vk[64];
  __shared__ double2 yk[64];
  const int g = glist[blockIdx.y];
  const BlockDev B = blocks[g];
  const int i = k + blockIdx.x;
  if (k >= B.ntiles || i >= B.ntiles) return;
  const int t = threadIdx.x, row = t >> 2, q = t & 3;
  double2* r = ws_at<double2>(ws, B.r_off);
  double2* y = ws_at<double2>(ws, B.y_off);
  if (t < 64) vk[t] = r[(int64_t)k * 64 + t];
  __syncthreads();
  const double2* Li = ws_at<double2>(ws, B.linv_off) + (int64_t)k * 4096;
  double2 s = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int e = 0; e < 16; ++e) s = cfma(Li[row * 64 + q * 16 + e], vk[q * 16 + e], s);
  s = quad_sum(s);
  if (q == 0) yk[row] = s;
  __syncthreads();
  if (i == k) {
    if (t < 64) y[(int64_t)k * 64 + t] = yk[t];
    return;
  }
  const double2* A = ws_at<double2>(ws, B.mat_off) + ((int64_t)i * 64) * B.m_pad + (int64_t)k * 64;
  s = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int e = 0; e < 16; ++e) s = cfma(A[(int64_t)row * B.m_pad + q * 16 + e], yk[q * 16 + e], s);
  s = quad_sum(s);
  if (q == 0) {
    const int64_t idx = (int64_t)i * 64 + row;
    r[idx] = csub(r[idx], s);
  }
}

__global__ void __launch_bounds__(256) k_trsv_bwd(const int32_t* glist, const BlockDev* blocks, char* ws, int k) {
  __shared__ double2 vk[64];
  __shared__ double2 ck[64];
  const int g = glist[blockIdx.y];
  const BlockDev B = blocks[g];
  if (k >= B.ntiles) return;
  const int i = k - (int)blockIdx.x;
  if (i < 0) return;
  const int t = threadIdx.x, col = t >> 2, q = t & 3;
  double2* y = ws_at<double2>(ws, B.y_off);
  if (t < 64) vk[t] = y[(int64_t)k * 64 + t];
  __syncthreads();
  const double2* Li = ws_at<double2>(ws, B.linv_off) + (int64_t)k * 4096;
  // c_k[col] = sum_r conj(Linv[r][col]) y_k[r]
  double2 s = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int e = 0; e < 16; ++e) {
    const int rr = q * 16 + e;
    s = cfmac(Li[rr * 64 + col], vk[rr], s);
  }
  s = quad_sum(s);
  if (q == 0) ck[col] = s;
  __syncthreads();
  if (i == k) {
    if (t < 64) {
      double2* x = ws_at<double2>(ws, B.x_off);
      const int64_t idx = (int64_t)k * 64 + t;
      x[idx] = cadd(x[idx], ck[t]);
    }
    return;
  }
  // y_i[col] -= sum_r conj(L_ki[r][col]) c_k[r]
  const double2* A = ws_at<double2>(ws, B.mat_off) + ((int64_t)k * 64) * B.m_pad + (int64_t)i * 64;
  s = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int e = 0; e < 16; ++e) {
    const int rr = q * 16 + e;
    s = cfmac(A[(int64_t)rr * B.m_pad + col], ck[rr], s);
  }
  s = quad_sum(s);
  if (q == 0) {
    const int64_t idx = (int64_t)i * 64 + col;
    y[idx] = csub(y[idx], s);
  }
}

// ---------------------------------------------------------------------------
void launch_potrf(const int32_t* glist, int n, const BlockDev* blocks, char* ws, int k, int32_t* status,
                  hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_potrf, dim3(n), dim3(256), 0, s, glist, blocks, ws, k, status);
}

void launch_tile_gemm(int mode, const TileTask* tasks, int n, const BlockDev* blocks, char* ws, int k, hipStream_t s) {
  if (n <= 0) return;
  if (mode == 0) hipLaunchKernelGGL(k_tile_gemm<0>, dim3(n), dim3(256), 0, s, tasks, blocks, ws, k);
  else hipLaunchKernelGGL(k_tile_gemm<1>, dim3(n), dim3(256), 0, s, tasks, blocks, ws, k);
}

void launch_trsv_fwd(const int32_t* glist, int n, int max_tiles_left, const BlockDev* blocks, char* ws, int k,
                     hipStream_t s) {
  if (n <= 0 || max_tiles_left <= 0) return;
  hipLaunchKernelGGL(k_trsv_fwd, dim3(max_tiles_left, n), dim3(256), 0, s, glist, blocks, ws, k);
}

void launch_trsv_bwd(const int32_t* glist, int n, int k, const BlockDev* blocks, char* ws, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_trsv_bwd, dim3(k + 1, n), dim3(256), 0, s, glist, blocks, ws, k);
}

}  // namespace qgt
