// Blocked Cholesky factorisation and triangular solves for the shifted block
// matrices (S_b + lambda I or the sample-space T_b + lambda I), batched over
// all blocks of all problems.  The matrices are Hermitian positive definite
// because lambda > 0, so the factorisation needs no pivoting.
//
// Storage: row-major m_pad x m_pad, lower triangle, 64x64 tiles, complex FP64,
// or complex FP32 where the plan factors a BF16-Gram block in FP32 (fact32);
// every kernel below takes its element type from the block it works on.
// Right-looking tile algorithm, step k:
//   POTRF  : L_kk L_kk^H = A_kk (one workgroup, in LDS) and Linv_kk = L_kk^{-1}
//   TRSM   : L_ik = A_ik Linv_kk^H                           (i > k)
//   UPDATE : A_ij -= L_ik L_jk^H                              (i >= j > k)
// Steps are taken in pairs: the update of column k+1 from panel k precedes
// step k+1, and the rest of the pair's trailing update reads both panels at
// once (K = 128), which halves the passes over the trailing matrix.
// TRSM and UPDATE are the same tile product C = beta C + alpha X Y^H on the
// matrix cores (v_mfma_f64_16x16x4_f64 or v_mfma_f32_16x16x4_f32, three real
// products per complex product).  Triangular solves use the stored Linv_kk for
// the diagonal tiles and accumulate in FP64 whatever the storage.
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

// Complex value (Re, Im) and MFMA accumulator of element type T.
template <typename T> using V2 = T __attribute__((ext_vector_type(2)));
template <typename T> using V4 = T __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4v mma4(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of the 16x16 MFMA result held by lane l in register r (its column is
// l % 16): 4 r + l / 16 for FP64, 4 (l / 16) + r for FP32.
template <typename T>
__device__ __forceinline__ int mma_row(int r, int lane) {
  return sizeof(T) == 8 ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}
// L_jj = sqrt(d) and 1 / L_jj for a pivot d > 0: correctly rounded FP64
// operations for an FP64 factor; the hardware reciprocal square root (about
// 1 ulp) for an FP32 factor, whose Gram carries BF16 rounding.
template <typename T>
__device__ __forceinline__ void pivot_sqrt(T d, T& ljj, T& inv) {
  if constexpr (sizeof(T) == 4) {
    inv = __builtin_amdgcn_rsqf(d);
    ljj = d * inv;
  } else if (d < 0x1p-1000) {  // far below the hardware estimate's range: the rounded library forms
    ljj = sqrt(d);
    inv = 1.0 / ljj;
  } else {
    // 1/sqrt(d) from the hardware estimate refined by two Newton steps
    // y <- y + y (1 - d y^2) / 2 (each at least doubles the correct bits), then
    // sqrt(d) = d y: ten dependent operations where the correctly rounded
    // square root and quotient take about thirty-five, on the serial chain of
    // pivots.  Both are within a few units in the last place.
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double e = fma(-d * y, y, 1.0);
      y = fma(0.5 * y, e, y);
    }
    inv = y;
    ljj = d * y;
  }
}
template <typename T>
__device__ __forceinline__ double2 to_c128(V2<T> v) {
  return make_double2((double)v.x, (double)v.y);
}

// ---------------------------------------------------------------------------
// POTRF of one 64x64 diagonal tile (lower triangle of A, leading dimension ld)
// by one 256-thread workgroup, plus X = L^{-1} written to Linv (64x64, dense
// with zeros above the diagonal).
//
// Blocked by 16 inside the tile.  For each diagonal block kb:
//   1. the workgroup factors the 16x16 diagonal block and inverts its factor,
//      one entry per thread, one barrier per column (chol16_wg);
//   2. the panel below is solved against it on the matrix cores,
//      P <- P D^{-H};
//   3. the trailing blocks are updated on the matrix cores, A_ij -= P_i P_j^H.
// L is written out, then the off-diagonal blocks of X = L^{-1} replace those
// of L in place, block column by block column from the right:
// X_ij = -sum_{j<p<=i} X_ip (L_pj D_j), with D_j = L_jj^{-1} and X_ii = D_i
// (from X L = I), also on the matrix cores.  Returns false if a pivot was not
// positive and finite (it is then replaced by 1 so that the factorisation
// terminates).
// Block-packed storage of the lower triangle of a 64x64 tile: the 10 blocks
// (ib, jb), jb <= ib, of 16x16 entries, each with row pitch 17, and the four
// inverses of the diagonal blocks: 61 KB in FP64, so that two workgroups fit
// on a CU (the persistent factorisation runs two per CU).
template <typename T> using Blk16 = V2<T>[16][17];
__device__ __forceinline__ int blk_index(int ib, int jb) { return ib * (ib + 1) / 2 + jb; }

template <typename T>
struct PotrfSmem {
  Blk16<T> L[10];  // the tile: A, then L, then (in place) the off-diagonal blocks of L^{-1}
  Blk16<T> D[4];   // inverses of the diagonal 16x16 blocks of L
};
union PotrfLds {
  PotrfSmem<double> d;
  PotrfSmem<float> f;
};

// 16x16 complex block product on the matrix cores by one wave:
//   NH: C = sum_t P[i][t] conj(Q[j][t])     NN: C = sum_t P[i][t] Q[t][j]
// Result in the MFMA layout (mma_row).
template <bool NH, typename T>
__device__ __forceinline__ void blk16_mma(const Blk16<T>& P, const Blk16<T>& Q, V4<T>& cr, V4<T>& ci) {
  const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int t = 4 * ks + kq;
    const V2<T> a = P[i][t];
    const V2<T> b = NH ? Q[i][t] : Q[t][i];
    if (NH) {  // a * conj(b)
      cr = mma4(a.x, b.x, cr);
      cr = mma4(a.y, b.y, cr);
      ci = mma4(a.y, b.x, ci);
      ci = mma4(-a.x, b.y, ci);
    } else {   // a * b
      cr = mma4(a.x, b.x, cr);
      cr = mma4(-a.y, b.y, cr);
      ci = mma4(a.y, b.x, ci);
      ci = mma4(a.x, b.y, ci);
    }
  }
}

// Workgroup-level Cholesky and inverse of the diagonal block (kb, kb), one
// entry per thread (thread = row * 16 + column): L into L, L^{-1} into D[kb]
// (both lower, zeros above).  Every thread reads the pivot and the column's
// entries at its row and its column from LDS, published by their owners at
// the end of the previous step into the other half of a double buffer, so
// that a step costs one workgroup barrier, one LDS latency and a few
// instructions per thread (a lone wave holding four entries per lane needs
// about 200 per step).  The
// inverse is built in the same steps by forward elimination, one step behind
// (row j of L^{-1} is final once scaled at step j): X_r -= L_rj X_j.
// Returns 2 * (pivots raised to the floor) + (1 if every pivot was finite),
// the same in every thread.
template <typename T>
struct Chol16Lds {
  V2<T> col[2][16];   // column j of the current block (the pivot at row j), by the parity of j
  V2<T> xrow[2][16];  // row j of the inverse
};

template <typename T>
__device__ __forceinline__ int chol16_wg(PotrfSmem<T>& sm, Chol16Lds<T>& cs, int kb, T floor) {
  const int t = threadIdx.x, r = t >> 4, c = t & 15;
  Blk16<T>& Tb = sm.L[blk_index(kb, kb)];
  Blk16<T>& Xb = sm.D[kb];
  V2<T> D = c <= r ? Tb[r][c] : V2<T>{0, 0};
  V2<T> X{c == r ? T(1) : T(0), T(0)};
  if (c == 0) cs.col[0][r] = D;
  int nfloor = 0;
  bool ok_all = true;
  V2<T> lprev{0, 0};  // L_r,j-1
  __syncthreads();
#pragma unroll 2
  for (int j = 0; j < 16; ++j) {
    const int b = j & 1;
    // the step's four LDS reads, issued together so that one latency is paid
    const T piv = cs.col[b][j].x;
    const V2<T> ar = cs.col[b][r];
    const V2<T> ac = cs.col[b][c];
    const V2<T> xj = cs.xrow[b ^ 1][c];  // row j - 1 of the inverse (unused at j = 0)
    // Every pivot of S + lambda I is at least lambda in exact arithmetic (a
    // pivot is the reciprocal of a diagonal entry of the inverse of a trailing
    // submatrix, whose eigenvalues are >= lambda).  A smaller pivot comes from
    // rounding (in the Gram, or in an FP32 factorisation) and is raised to
    // lambda: the factor is then that of a nearby positive definite matrix,
    // which is all the preconditioner needs.  NaN or infinity fails.
    T d = piv;
    const bool ok = d == d && d < T(INFINITY);
    if (!ok) d = T(1);
    else if (!(d >= floor)) {
      d = floor;
      ++nfloor;  // the pivot is the same in every thread
    }
    ok_all &= ok;
    T ljj, inv;
    pivot_sqrt<T>(d, ljj, inv);
    const V2<T> lrj = r > j ? ar * inv : V2<T>{0, 0};
    if (c == j) {
      if (r >= j) D = r > j ? lrj : V2<T>{ljj, T(0)};
    } else if (c > j && c <= r) {
      const V2<T> lcj = ac * inv;
      D = V2<T>{D.x - (lrj.x * lcj.x + lrj.y * lcj.y), D.y - (lrj.y * lcj.x - lrj.x * lcj.y)};
    }
    // the inverse: row j - 1 (final since the last step) eliminated from the
    // rows below, then row j scaled and published
    if (j > 0 && r >= j && c < j)
      X = V2<T>{X.x - (lprev.x * xj.x - lprev.y * xj.y), X.y - (lprev.x * xj.y + lprev.y * xj.x)};
    if (r == j) {
      X = X * inv;
      cs.xrow[b][c] = X;
    }
    // column j + 1 for the next step
    if (j + 1 < 16 && c == j + 1) cs.col[b ^ 1][r] = D;
    lprev = lrj;
    __syncthreads();
  }
  Tb[r][c] = c <= r ? D : V2<T>{0, 0};
  Xb[r][c] = c <= r ? X : V2<T>{0, 0};
  return 2 * nfloor + (ok_all ? 1 : 0);
}

// Store a 16x16 block result (MFMA layout) into LDS, scaled by s.
template <typename T>
__device__ __forceinline__ void blk16_store(Blk16<T>& dst, const V4<T>& cr, const V4<T>& ci, T s) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[mma_row<T>(q, lane)][lane & 15] = V2<T>{s * cr[q], s * ci[q]};
}

template <typename T>
__device__ bool potrf_tile(V2<T>* A, int64_t ld, V2<T>* Linv, PotrfSmem<T>& sm, T floor, int* s_floors) {
  const int t = threadIdx.x, w = t >> 6;
  {
    // all ten loads of this thread in flight together, then the LDS stores
    constexpr int kIb[10] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
    constexpr int kJb[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
    const int r = t >> 4, c = t & 15;
    V2<T> v[10];
#pragma unroll
    for (int bk = 0; bk < 10; ++bk) {
      const int i = 16 * kIb[bk] + r, j = 16 * kJb[bk] + c;
      v[bk] = j <= i ? ((const QGT_GLOBAL V2<T>*)A)[(int64_t)i * ld + j] : V2<T>{0, 0};
    }
#pragma unroll
    for (int bk = 0; bk < 10; ++bk) sm.L[bk][r][c] = v[bk];
  }
  __shared__ int s_ok;
  if (t == 0) {
    s_ok = 1;
    *s_floors = 0;
  }
  __syncthreads();
  __shared__ Chol16Lds<T> cs;
  for (int kb = 0; kb < 4; ++kb) {
    {
      const int r = chol16_wg<T>(sm, cs, kb, floor);
      if (t == 0) {
        if (!(r & 1)) s_ok = 0;
        *s_floors += r >> 1;
      }
    }
    __syncthreads();
    // panel solve P_ib <- P_ib D^{-H}, one block row per wave
    for (int ib = kb + 1 + w; ib < 4; ib += 4) {
      V4<T> cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
      blk16_mma<true, T>(sm.L[blk_index(ib, kb)], sm.D[kb], cr, ci);
      __builtin_amdgcn_wave_barrier();
      blk16_store<T>(sm.L[blk_index(ib, kb)], cr, ci, T(1));
    }
    __syncthreads();
    // trailing update A_(ib,jb) -= P_ib P_jb^H, kb < jb <= ib < 4
    int task = 0;
    for (int ib = kb + 1; ib < 4; ++ib)
      for (int jb = kb + 1; jb <= ib; ++jb, ++task) {
        if ((task & 3) != w) continue;
        V4<T> cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
        blk16_mma<true, T>(sm.L[blk_index(ib, kb)], sm.L[blk_index(jb, kb)], cr, ci);
        Blk16<T>& C = sm.L[blk_index(ib, jb)];
        const int lane = t & 63;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          V2<T>& e = C[mma_row<T>(q, lane)][lane & 15];
          e = V2<T>{e.x - cr[q], e.y - ci[q]};
        }
      }
    __syncthreads();
  }
  // the factor, before its off-diagonal blocks are overwritten by the inverse
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    if (j <= i) A[(int64_t)i * ld + j] = sm.L[blk_index(i >> 4, j >> 4)][i & 15][j & 15];
  }
  __syncthreads();
  // X = L^{-1} in place, block columns jb = 2, 1, 0: first W_p = L_p,jb D_jb
  // (p > jb, in place, one block per wave), then X_ib,jb = -sum_{jb<p<=ib}
  // X_ib,p W_p with X_ib,ib = D_ib and X_ib,p (p < ib) already in place; the
  // results stay in registers until every wave has read the W_p.
#pragma unroll
  for (int jb = 2; jb >= 0; --jb) {
    if (jb + 1 + w < 4) {  // W_p for p = jb + 1 + w
      const int p = jb + 1 + w;
      V4<T> cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
      blk16_mma<false, T>(sm.L[blk_index(p, jb)], sm.D[jb], cr, ci);
      __builtin_amdgcn_wave_barrier();
      blk16_store<T>(sm.L[blk_index(p, jb)], cr, ci, T(1));
    }
    __syncthreads();
    const int ib = jb + 1 + w;
    V4<T> cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    if (ib < 4) {
#pragma unroll
      for (int p = jb + 1; p < 4; ++p)
        if (p <= ib) blk16_mma<false, T>(p == ib ? sm.D[p] : sm.L[blk_index(ib, p)], sm.L[blk_index(p, jb)], cr, ci);
    }
    __syncthreads();
    if (ib < 4) blk16_store<T>(sm.L[blk_index(ib, jb)], cr, ci, T(-1));
    __syncthreads();
  }
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    const int ib = i >> 4, jb = j >> 4;
    Linv[idx] = j > i ? V2<T>{0, 0} : (ib == jb ? sm.D[ib][i & 15][j & 15] : sm.L[blk_index(ib, jb)][i & 15][j & 15]);
  }
  return s_ok != 0;
}

__global__ void __launch_bounds__(256) k_potrf(const int32_t* glist, const BlockDev* blocks, char* ws, int k,
                                               int32_t* status, int32_t* floors) {
  __shared__ PotrfLds sm;
  __shared__ int s_floors;
  const int g = glist[blockIdx.x];
  const BlockDev B = blocks[g];
  if (k >= B.ntiles) return;
  const int64_t a0 = ((int64_t)k * 64) * B.m_pad + (int64_t)k * 64;
  bool ok;
  if (B.fact32)
    ok = potrf_tile<float>(ws_at<V2<float>>(ws, B.mat_off) + a0, B.m_pad,
                           ws_at<V2<float>>(ws, B.linv_off) + (int64_t)k * 4096, sm.f, (float)B.lambda, &s_floors);
  else
    ok = potrf_tile<double>(ws_at<V2<double>>(ws, B.mat_off) + a0, B.m_pad,
                            ws_at<V2<double>>(ws, B.linv_off) + (int64_t)k * 4096, sm.d, B.lambda, &s_floors);
  if (threadIdx.x == 0) {
    if (!ok) status[g] = 5;  // QGT_ERR_NOT_POSITIVE_DEFINITE (NaN or infinite pivot)
    if (s_floors) atomicAdd(&floors[g], s_floors);
  }
}

// ---------------------------------------------------------------------------
// Tile product on the matrix cores: C = X Y^H (MODE 0) or C -= X Y^H (MODE 1)
// for 64x64 tiles, K = kGemmSW * nst in LDS stages of kGemmSW columns.  Complex
// product with three real MFMA products (Gauss), X = a + ib, Y = c + id:
//   Re(X Y^H) = a c^T + b d^T,  Im(X Y^H) = (a + b)(c - d)^T - a c^T + b d^T.
// C may alias X (TRSM in place): every read of X precedes the first write.
// Stages of 8 columns keep the workgroup at 18 KB of LDS in FP64, so that a
// POTRF workgroup (87.5 KB) still fits on a CU that runs four of them.
constexpr int kGemmSW = 8;
template <typename T>
struct GemmSmem {
  V2<T> Xs[64][kGemmSW + 1];
  V2<T> Ys[64][kGemmSW + 1];
};
union GemmLds {
  GemmSmem<double> d;
  GemmSmem<float> f;
};

template <int MODE, typename T>
__device__ void tile_gemm_nh(V2<T>* Cp, int64_t ldc, const V2<T>* Xp, int64_t ldx, const V2<T>* Yp, int64_t ldy,
                             int NST, GemmSmem<T>& sm) {
  constexpr int SW = kGemmSW, PER = SW / 4;  // PER complex loads per thread and stage
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1, l16 = lane & 15;
  // P1 = a c^T, P2 = b d^T, P3 = (a + b)(c - d)^T: Re = P1 + P2, Im = P3 - P1 + P2
  V4<T> acc1[2][2], acc2[2][2], acc3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { acc1[a][b][r] = 0; acc2[a][b][r] = 0; acc3[a][b][r] = 0; }
  // operand staging: the loads of a stage are issued together, and the next
  // stage's loads are in flight while the current stage computes
  const int lrow = t >> 2, lq = t & 3, lg = lane >> 4;
  const V2<T>* Xv = Xp + (int64_t)lrow * ldx + lq * PER;
  const V2<T>* Yv = Yp + (int64_t)lrow * ldy + lq * PER;
  V2<T> xv[PER], yv[PER];
#pragma unroll
  for (int e = 0; e < PER; ++e) {
    xv[e] = Xv[e];
    yv[e] = Yv[e];
  }
  for (int st = 0; st < NST; ++st) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      sm.Xs[lrow][lq * PER + e] = xv[e];
      sm.Ys[lrow][lq * PER + e] = yv[e];
    }
    __syncthreads();
    if (st + 1 < NST) {
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        xv[e] = Xv[(st + 1) * SW + e];
        yv[e] = Yv[(st + 1) * SW + e];
      }
    }
#pragma unroll
    for (int e = 0; e < SW / 4; ++e) {
      const int kk = (SW / 4) * lg + e;
      V2<T> xa[2], yb[2];
      T xs[2], yd[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        xa[s] = sm.Xs[32 * wr + 16 * s + l16][kk];
        yb[s] = sm.Ys[32 * wc + 16 * s + l16][kk];
        xs[s] = xa[s].x + xa[s].y;
        yd[s] = yb[s].x - yb[s].y;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc1[a][b] = mma4(xa[a].x, yb[b].x, acc1[a][b]);
          acc2[a][b] = mma4(xa[a].y, yb[b].y, acc2[a][b]);
          acc3[a][b] = mma4(xs[a], yd[b], acc3[a][b]);
        }
    }
  }
  __syncthreads();  // all reads of X (possibly aliased with C) are done
  V2<T> old[2][2][4];
  if (MODE == 1) {  // every old value is loaded before the first store
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          old[a][b][r] = Cp[(int64_t)(32 * wr + 16 * a + mma_row<T>(r, lane)) * ldc + 32 * wc + 16 * b + l16];
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        V2<T>* c = Cp + (int64_t)(32 * wr + 16 * a + mma_row<T>(r, lane)) * ldc + 32 * wc + 16 * b + l16;
        const V2<T> v{acc1[a][b][r] + acc2[a][b][r], acc3[a][b][r] - acc1[a][b][r] + acc2[a][b][r]};
        *c = MODE == 0 ? v : old[a][b][r] - v;
      }
}

// ---------------------------------------------------------------------------
// Tile tasks of the right-looking Cholesky:
//   MODE 0 (TRSM)  : L_ik = A_ik Linv_kk^H, in place
//   MODE 1 (UPDATE): A_ij -= L_ik L_jk^H                          (K = 64)
//   MODE 2 (UPDATE): A_ij -= L_ik L_jk^H + L_i,k+1 L_j,k+1^H      (K = 128, the
//                    two adjacent panels of a pair of steps read as one)
template <int MODE, typename T>
__device__ __forceinline__ void tile_task(const int4 tk, const BlockDev& B, char* ws, int k, GemmSmem<T>& sm) {
  const int64_t ld = B.m_pad;
  V2<T>* Abase = ws_at<V2<T>>(ws, B.mat_off);
  V2<T>* Cp = Abase + ((int64_t)tk.y * 64) * ld + (int64_t)tk.z * 64;
  const V2<T>* Xp = Abase + ((int64_t)tk.y * 64) * ld + (int64_t)k * 64;
  if (MODE == 0)
    tile_gemm_nh<0, T>(Cp, ld, Xp, ld, ws_at<V2<T>>(ws, B.linv_off) + (int64_t)k * 4096, 64, 64 / kGemmSW, sm);
  else if (MODE == 1)
    tile_gemm_nh<1, T>(Cp, ld, Xp, ld, Abase + ((int64_t)tk.z * 64) * ld + (int64_t)k * 64, ld, 64 / kGemmSW, sm);
  else tile_gemm_nh<1, T>(Cp, ld, Xp, ld, Abase + ((int64_t)tk.z * 64) * ld + (int64_t)k * 64, ld, 128 / kGemmSW, sm);
}

// One kernel serves both factor types.  Its register use (about 180 per lane,
// set by the FP64 path) holds it to two workgroups per CU, which leaves room
// on every CU for a POTRF workgroup (87.5 KB of LDS, about 136 registers)
// beside the large lookahead updates.  Separate FP32 kernels (110 registers,
// four workgroups per CU) made the updates 15-20% faster but left POTRF
// waiting for them to drain (56 -> 131 us) and the factorisation slower.
template <int MODE>
__global__ void __launch_bounds__(256, 2) k_tile_gemm(const int4* tasks, const BlockDev* blocks, char* ws, int k) {
  __shared__ GemmLds sm;
  const int4 tk = tasks[blockIdx.x];
  const BlockDev B = blocks[tk.x];
  if (B.fact32) tile_task<MODE, float>(tk, B, ws, k, sm.f);
  else tile_task<MODE, double>(tk, B, ws, k, sm.d);
}

// ---------------------------------------------------------------------------
constexpr int kSpinLimit = 1 << 22;

// Ticket for the calling workgroup.  The value is made wave-uniform
// (readfirstlane) so that every branch and loop that depends on it is a scalar
// branch: a loop around a ticket must never be compiled with a divergent exit,
// because thread 0 (which takes the next ticket) would leave it before the
// other lanes.  Also clears the workgroup's failure flag.
__device__ __forceinline__ int take_ticket(int* counter, int* s_ticket, int* s_fail) {
  __syncthreads();
  if (threadIdx.x == 0) {
    *s_fail = 0;
    *s_ticket = atomicAdd(counter, 1);
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(*s_ticket);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Thread 0 waits until *flag >= target (bounded); on expiry *s_fail is set.
__device__ __forceinline__ void spin_ge(const int* flag, int target, int* s_fail) {
  int spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > kSpinLimit) {
      *s_fail = 1;
      return;
    }
  }
}

// ---------------------------------------------------------------------------
// The Cholesky of every block of the plan as one persistent launch.
//
// The host lists the tile tasks of all blocks (CholTask: POTRF, TRSM and the
// trailing updates in chunks of panels) in an order that is topological for
// every block's dependency graph, by decreasing length of the longest path to
// the end of the factorisation (critical path first across all blocks), and
// splits it into one ticket queue per XCD: every operation on tile (i, j) of
// block g runs on XCD chol_owner(g, i, j).  Each workgroup reads the id of the
// XCD it runs on from the hardware and takes the next task of that XCD's queue
// by ticket, then waits until the tiles it reads are final and every earlier
// operation on its own tile is done.  A task waits only for tasks earlier in
// the global order; those are in its own queue at smaller tickets (held or
// finished by workgroups that started earlier) or in other queues, whose
// progress does not depend on it, so the waits end however many workgroups are
// resident.  Each wait is bounded, and after one has given up (status
// QGT_ERR_INTERNAL) every other wait returns at once so that the launch always
// drains.
//
// Memory ordering.  The XCDs have separate L2 caches.  A tile's intermediate
// values (before its final operation) are read and written only on its owner
// XCD, through that XCD's L2: an update publishes them by waiting for its
// stores to complete, and a consumer on the same XCD invalidates its CU's L1
// (device-scope acquire) before reading.  A final tile is read on every XCD: its POTRF or TRSM takes a
// device-scope release fence (the XCD's L2 written back) before publishing,
// and no other XCD can hold a stale copy of it, since no other XCD reads a
// tile before it is final and every workgroup takes a device-scope acquire
// fence when it starts (clearing copies left by earlier launches).  Final
// tiles then stay in each reader's L2 for the many tasks that read them.
// Counters are device-scope atomics.
union CholLds {
  PotrfSmem<double> pd;
  PotrfSmem<float> pf;
  GemmSmem<double> gd;
  GemmSmem<float> gf;
};

// Wave 0 waits for the task's dependencies (lane l polls condition l).
__device__ __forceinline__ void chol_wait(const CholTask& tk, const BlockDev& B, const int* state, int* abort_flag,
                                          int* s_fail) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int c = B.chunk;
  const int* st = state + B.tile_state;
  int idx = -1, target = 0;
  if (tk.type == CHOL_UPD) {
    const int n = tk.k1 - tk.k0;
    if (lane == 0) {
      idx = tri_index(tk.i, tk.j);
      target = kCholWaves * tk.seq;
    } else if (lane <= n) {
      const int k = tk.k0 + lane - 1;
      idx = tri_index(tk.i, k);
      target = kCholWaves * (chol_nchunks(k, c) + 1);
    } else if (lane <= 2 * n) {
      const int k = tk.k0 + lane - n - 1;
      idx = tri_index(tk.j, k);
      target = kCholWaves * (chol_nchunks(k, c) + 1);
    }
  } else if (tk.type == CHOL_TRSM) {
    if (lane == 0) {
      idx = tri_index(tk.i, tk.j);
      target = kCholWaves * tk.seq;
    } else if (lane == 1) {
      idx = tri_index(tk.j, tk.j);
      target = kCholWaves * (tk.seq + 1);
    }
  } else if (lane == 0) {
    idx = tri_index(tk.i, tk.i);
    target = kCholWaves * tk.seq;
  }
  int spins = 0;
  for (;;) {
    const int v = idx >= 0 ? __hip_atomic_load(st + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : target;
    if (__all(v >= target)) break;
    if (uniform(__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0) {
      if (lane == 0) *s_fail = 1;
      break;
    }
    if (++spins > kSpinLimit) {
      if (lane == 0) {
        *s_fail = 1;
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

template <typename T>
__device__ __forceinline__ void chol_run(const CholTask& tk, const BlockDev& B, char* ws, CholLds& sm,
                                         PotrfSmem<T>& psm, GemmSmem<T>& gsm, int* s_floors, int* s_bad) {
  const int64_t ld = B.m_pad;
  V2<T>* A = ws_at<V2<T>>(ws, B.mat_off);
  V2<T>* Linv = ws_at<V2<T>>(ws, B.linv_off);
  if (tk.type == CHOL_POTRF) {
    const int k = tk.i;
    const bool ok = potrf_tile<T>(A + ((int64_t)k * 64) * ld + (int64_t)k * 64, ld, Linv + (int64_t)k * 4096, psm,
                                  (T)B.lambda, s_floors);
    if (threadIdx.x == 0 && !ok) *s_bad = 1;
  } else if (tk.type == CHOL_TRSM) {
    V2<T>* C = A + ((int64_t)tk.i * 64) * ld + (int64_t)tk.j * 64;
    tile_gemm_nh<0, T>(C, ld, C, ld, Linv + (int64_t)tk.j * 4096, 64, 64 / kGemmSW, gsm);
  } else {
    tile_gemm_nh<1, T>(A + ((int64_t)tk.i * 64) * ld + (int64_t)tk.j * 64, ld,
                       A + ((int64_t)tk.i * 64) * ld + (int64_t)tk.k0 * 64, ld,
                       A + ((int64_t)tk.j * 64) * ld + (int64_t)tk.k0 * 64, ld, (tk.k1 - tk.k0) * 64 / kGemmSW, gsm);
  }
}

// XCD of the calling workgroup (the XCC_ID hardware register), modulo nq.
__device__ __forceinline__ int xcd_id(int nq) {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & 0xF) % nq;
}

// ctl[q]: ticket counter of XCD queue q, ctl[8]: abort flag (all zero before
// the launch).  qoff[q] .. qoff[q + 1]: the tasks of queue q.
__global__ void __launch_bounds__(256, 2) k_chol(const CholTask* tasks, const int32_t* qoff, int nq,
                                                 const BlockDev* blocks, char* ws, int* state, int* ctl,
                                                 int32_t* status, int32_t* floors) {
  __shared__ CholLds sm;
  __shared__ int s_ticket, s_fail, s_floors, s_bad;
  const int q = uniform(xcd_id(nq));
  const int q0 = uniform(qoff[q]), qn = uniform(qoff[q + 1] - qoff[q]);
  // drop copies of tiles cached by earlier launches
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (;;) {
    const int t = take_ticket(&ctl[q], &s_ticket, &s_fail);  // also clears s_fail
    if (t >= qn) break;
    if (threadIdx.x == 0) {
      s_floors = 0;
      s_bad = 0;
    }
    const CholTask tk = tasks[q0 + t];
    const int g = uniform(tk.g);
    const BlockDev B = blocks[g];
    chol_wait(tk, B, state, &ctl[8], &s_fail);
    __syncthreads();
    // this CU's L1 may hold older values of the tiles this task reads (an
    // earlier task on the same tile may have run on this CU): every wave
    // invalidates it before its own first load.  This takes the device-scope
    // acquire: a workgroup-scope invalidate does nothing when a workgroup
    // runs on one CU, since the L1 is then coherent at that scope.
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (uniform(B.fact32)) chol_run<float>(tk, B, ws, sm, sm.pf, sm.gf, &s_floors, &s_bad);
    else chol_run<double>(tk, B, ws, sm, sm.pd, sm.gd, &s_floors, &s_bad);
    // publish the tile: every wave waits for its own stores (a final tile is
    // also written back from this XCD's L2), then counts itself
    if (tk.type == CHOL_UPD) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0)
      __hip_atomic_fetch_add(state + B.tile_state + tri_index(tk.i, tk.j), 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_fail) status[g] = 8;        // QGT_ERR_INTERNAL: a bounded wait gave up
      else if (s_bad) status[g] = 5;    // QGT_ERR_NOT_POSITIVE_DEFINITE (NaN or infinite pivot)
      if (s_floors) atomicAdd(&floors[g], s_floors);
    }
  }
}

// ---------------------------------------------------------------------------
// Triangular solves, one persistent launch per solve for all listed blocks.
//
// Each workgroup takes a ticket; tickets enumerate the tiles of every block in
// dependency order (forward: tile 0, 1, ...; backward: the last tile first).  A
// tile waits only for tiles of the same block with smaller tickets, which
// belong to workgroups that started earlier, so the waits end whatever the
// number of resident workgroups.  Each wait is bounded (QGT_ERR_INTERNAL in
// status on expiry), so the kernel always exits.
//
// The vectors exchanged between workgroups (64 entries per tile) carry their
// own readiness: before the solve every 64-bit word of them holds kEmpty, a
// signalling-NaN pattern that no arithmetic result can take (results and
// propagated NaNs are quiet); a producer writes each word once with a
// device-scope atomic store, and a consumer wave polls the words it needs until
// none is kEmpty.  No flag, no release fence and no wait for store completion
// is needed, which keeps one step of the dependency chain to about one store
// and one load through the device-coherent level.  The matrix tiles, written
// by earlier launches, are read with ordinary loads, issued before the wait.
//
// Forward  (L y = r): y_i = Linv_ii (r_i - sum_{j<i} L_ij y_j)
// Backward (L^H z = y): z_i = Linv_ii^H (y_i - sum_{j>i} L_ji^H z_j), so that
// z = M^{-1} r with M = L L^H.
constexpr unsigned long long kEmpty = 0x7FF00000DEAD0001ull;

__device__ __forceinline__ double2 quad_sum(double2 v) {
  v.x += __shfl_xor(v.x, 1, 64);
  v.y += __shfl_xor(v.y, 1, 64);
  v.x += __shfl_xor(v.x, 2, 64);
  v.y += __shfl_xor(v.y, 2, 64);
  return v;
}

__device__ __forceinline__ void store_dev(double2* p, double2 v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One whole wave polls one complex entry per lane until every lane's entry has
// been written (bounded; on expiry *s_fail is set and the stale value returned).
// The exit test is a wave vote, so the loop is uniform.
__device__ __forceinline__ double2 poll_dev(const double2* p, int* s_fail) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(const_cast<double2*>(p));
  unsigned long long a, b;
  int spins = 0;
  for (;;) {
    a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__all(a != kEmpty && b != kEmpty)) break;
    if (++spins > kSpinLimit) {
      if ((threadIdx.x & 63) == 0) *s_fail = 1;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}

// As poll_dev for two entries per lane (two consecutive tiles).
__device__ __forceinline__ void poll2_dev(const double2* p0, const double2* p1, double2& v0, double2& v1,
                                          int* s_fail) {
  unsigned long long* q0 = reinterpret_cast<unsigned long long*>(const_cast<double2*>(p0));
  unsigned long long* q1 = reinterpret_cast<unsigned long long*>(const_cast<double2*>(p1));
  unsigned long long a, b, c, d;
  int spins = 0;
  for (;;) {
    a = __hip_atomic_load(q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b = __hip_atomic_load(q0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    c = __hip_atomic_load(q1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    d = __hip_atomic_load(q1 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__all(a != kEmpty && b != kEmpty && c != kEmpty && d != kEmpty)) break;
    if (++spins > kSpinLimit) {
      if ((threadIdx.x & 63) == 0) *s_fail = 1;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  v0 = make_double2(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
  v1 = make_double2(__longlong_as_double((long long)c), __longlong_as_double((long long)d));
}

// Marks the exchanged vectors y and z of every block empty (m_pad entries each).
__global__ void __launch_bounds__(256) k_trsv_reset(const BlockDev* blocks, char* ws) {
  const BlockDev B = blocks[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  // a converged block keeps its last correction z for the final CG step
  if (i >= 2 * B.m_pad || cg_done(B, ws)) return;
  unsigned long long* y = ws_at<unsigned long long>(ws, B.y_off);
  unsigned long long* z = ws_at<unsigned long long>(ws, B.z_off);
  y[i] = kEmpty;
  z[i] = kEmpty;
}

// Index of entry i (0..63) of an exchanged 64-entry vector in LDS: groups of
// 16 are 17 entries apart, so that the four entries a wave reads at once
// (one per group) fall in different banks.
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Forward solve of tile i of block B (the kernel below holds the ticket).
template <typename T>
__device__ __forceinline__ void trsv_fwd_tile(const BlockDev& B, char* ws, int i, double2* vj, double2* vj2,
                                              int* s_fail) {
  const int t = threadIdx.x, row = t >> 2, q = t & 3;
  const V2<T>* Arow = ws_at<V2<T>>(ws, B.mat_off) + ((int64_t)i * 64 + row) * B.m_pad + q * 16;
  double2* y = ws_at<double2>(ws, B.y_off);
  const double2* r = ws_at<double2>(ws, B.r_off);
  // the diagonal inverse and the right-hand side do not depend on other
  // tiles: load them first, off the dependency chain
  const V2<T>* Li = ws_at<V2<T>>(ws, B.linv_off) + (int64_t)i * 4096 + row * 64 + q * 16;
  V2<T> Lip[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) Lip[e] = Li[e];
  const double2 rv = r[(int64_t)i * 64 + row];
  double2 acc = make_double2(0.0, 0.0);
  V2<T> Lt[16], Lt2[16];
  // two tiles per iteration: one round trip to memory covers both (the tiles
  // far behind the front of the solve are ready and only stream)
  int j = 0;
  for (; j + 1 < i; j += 2) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      Lt[e] = Arow[(int64_t)j * 64 + e];
      Lt2[e] = Arow[(int64_t)(j + 1) * 64 + e];
    }
    if (t < 64) poll2_dev(y + (int64_t)j * 64 + t, y + (int64_t)(j + 1) * 64 + t, vj[pad16(t)], vj2[pad16(t)], s_fail);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfma(to_c128<T>(Lt[e]), vj[q * 17 + e], acc);
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfma(to_c128<T>(Lt2[e]), vj2[q * 17 + e], acc);
    __syncthreads();
  }
  if (j < i) {
#pragma unroll
    for (int e = 0; e < 16; ++e) Lt[e] = Arow[(int64_t)j * 64 + e];
    if (t < 64) vj[pad16(t)] = poll_dev(y + (int64_t)j * 64 + t, s_fail);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfma(to_c128<T>(Lt[e]), vj[q * 17 + e], acc);
    __syncthreads();
  }
  acc = quad_sum(acc);
  if (q == 0) vj[pad16(row)] = csub(rv, acc);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 16; ++e) s = cfma(to_c128<T>(Lip[e]), vj[q * 17 + e], s);
  s = quad_sum(s);
  if (q == 0) store_dev(y + (int64_t)i * 64 + row, s);
}

__global__ void __launch_bounds__(256) k_trsv_fwd(const int2* tmap, int ntickets, const BlockDev* blocks, char* ws,
                                                  int* counter, int32_t* status) {
  __shared__ double2 vj[68], vj2[68];
  __shared__ int s_ticket, s_fail;
  const int tk = take_ticket(counter, &s_ticket, &s_fail);
  if (tk >= ntickets) return;
  const int g = uniform(tmap[tk].x), i = uniform(tmap[tk].y);
  const BlockDev B = blocks[g];
  if (uniform(cg_done(B, ws))) return;  // every tile of a converged block is skipped
  if (uniform(B.fact32)) trsv_fwd_tile<float>(B, ws, i, vj, vj2, &s_fail);
  else trsv_fwd_tile<double>(B, ws, i, vj, vj2, &s_fail);
  if (threadIdx.x == 0 && s_fail) status[g] = 8;  // QGT_ERR_INTERNAL
}

// Backward solve of tile i of block B.
template <typename T>
__device__ __forceinline__ void trsv_bwd_tile(const BlockDev& B, char* ws, int i, double2* vj, double2* vj2,
                                              int* s_fail) {
  const int t = threadIdx.x, col = t >> 2, q = t & 3;
  const V2<T>* Abase = ws_at<V2<T>>(ws, B.mat_off);
  // y is complete: this launch starts after the forward solve has finished
  const double2* y = ws_at<double2>(ws, B.y_off);
  double2* c = ws_at<double2>(ws, B.z_off);
  const V2<T>* Li = ws_at<V2<T>>(ws, B.linv_off) + (int64_t)i * 4096 + (q * 16) * 64 + col;
  V2<T> Lip[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) Lip[e] = Li[e * 64];
  const double2 yv = y[(int64_t)i * 64 + col];
  double2 acc = make_double2(0.0, 0.0);
  V2<T> Lt[16], Lt2[16];
  int j = B.ntiles - 1;
  for (; j - 1 > i; j -= 2) {
    // column col of tiles L_ji and L_j-1,i, rows q*16 .. q*16+15
    const V2<T>* Lji = Abase + ((int64_t)j * 64 + q * 16) * B.m_pad + (int64_t)i * 64 + col;
    const V2<T>* Lj2 = Lji - 64 * B.m_pad;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      Lt[e] = Lji[(int64_t)e * B.m_pad];
      Lt2[e] = Lj2[(int64_t)e * B.m_pad];
    }
    if (t < 64) poll2_dev(c + (int64_t)j * 64 + t, c + (int64_t)(j - 1) * 64 + t, vj[pad16(t)], vj2[pad16(t)], s_fail);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfmac(to_c128<T>(Lt[e]), vj[q * 17 + e], acc);
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfmac(to_c128<T>(Lt2[e]), vj2[q * 17 + e], acc);
    __syncthreads();
  }
  if (j > i) {
    const V2<T>* Lji = Abase + ((int64_t)j * 64 + q * 16) * B.m_pad + (int64_t)i * 64 + col;
#pragma unroll
    for (int e = 0; e < 16; ++e) Lt[e] = Lji[(int64_t)e * B.m_pad];
    if (t < 64) vj[pad16(t)] = poll_dev(c + (int64_t)j * 64 + t, s_fail);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) acc = cfmac(to_c128<T>(Lt[e]), vj[q * 17 + e], acc);
    __syncthreads();
  }
  acc = quad_sum(acc);
  if (q == 0) vj[pad16(col)] = csub(yv, acc);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int e = 0; e < 16; ++e) s = cfmac(to_c128<T>(Lip[e]), vj[q * 17 + e], s);
  s = quad_sum(s);
  if (q == 0) store_dev(c + (int64_t)i * 64 + col, s);
}

__global__ void __launch_bounds__(256) k_trsv_bwd(const int2* tmap, int ntickets, const BlockDev* blocks, char* ws,
                                                  int* counter, int32_t* status) {
  __shared__ double2 vj[68], vj2[68];
  __shared__ int s_ticket, s_fail;
  const int tk = take_ticket(counter, &s_ticket, &s_fail);
  if (tk >= ntickets) return;
  const int g = uniform(tmap[tk].x), i = uniform(tmap[tk].y);
  const BlockDev B = blocks[g];
  if (uniform(cg_done(B, ws))) return;  // every tile of a converged block is skipped
  if (uniform(B.fact32)) trsv_bwd_tile<float>(B, ws, i, vj, vj2, &s_fail);
  else trsv_bwd_tile<double>(B, ws, i, vj, vj2, &s_fail);
  if (threadIdx.x == 0 && s_fail) status[g] = 8;  // QGT_ERR_INTERNAL
}

// ---------------------------------------------------------------------------
void launch_potrf(const int32_t* glist, int n, const BlockDev* blocks, char* ws, int k, int32_t* status,
                  int32_t* floors, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_potrf, dim3(n), dim3(256), 0, s, glist, blocks, ws, k, status, floors);
}

void launch_tile_gemm(int mode, const int4* tasks, int n, const BlockDev* blocks, char* ws, int k, hipStream_t s) {
  if (n <= 0) return;
  if (mode == 0) hipLaunchKernelGGL(k_tile_gemm<0>, dim3(n), dim3(256), 0, s, tasks, blocks, ws, k);
  else if (mode == 1) hipLaunchKernelGGL(k_tile_gemm<1>, dim3(n), dim3(256), 0, s, tasks, blocks, ws, k);
  else hipLaunchKernelGGL(k_tile_gemm<2>, dim3(n), dim3(256), 0, s, tasks, blocks, ws, k);
}

void launch_chol(const CholTask* tasks, const int32_t* qoff, int nq, int ntasks, int nwg, const BlockDev* blocks,
                 char* ws, int* state, int* ctl, int32_t* status, int32_t* floors, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_chol, dim3(nwg), dim3(256), 0, s, tasks, qoff, nq, blocks, ws, state, ctl, status, floors);
}

void launch_trsv_reset(const BlockDev* blocks, char* ws, int nblocks, int64_t max_mpad, hipStream_t s) {
  hipLaunchKernelGGL(k_trsv_reset, dim3((unsigned)((2 * max_mpad + 255) / 256), nblocks), dim3(256), 0, s, blocks, ws);
}

void launch_trsv(int dir, const int2* tmap, int ntickets, const BlockDev* blocks, char* ws, int* counter,
                 int32_t* status, hipStream_t s) {
  if (ntickets <= 0) return;
  if (dir == 0)
    hipLaunchKernelGGL(k_trsv_fwd, dim3(ntickets), dim3(256), 0, s, tmap, ntickets, blocks, ws, counter, status);
  else
    hipLaunchKernelGGL(k_trsv_bwd, dim3(ntickets), dim3(256), 0, s, tmap, ntickets, blocks, ws, counter, status);
}

}  // namespace qgt
