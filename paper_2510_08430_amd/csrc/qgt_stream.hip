// Streaming (HBM-bound) kernels of the block-SR path for gfx950:
//   * binding of the per-call pointers,
//   * centred local energy (Eq. 1 estimated over the samples),
//   * the column pass over O: column means and force (Eq. 2 centring, force
//     dO^H dE / n_s), and the column half of the matrix-free refinement
//     residual and of the sample-space back-projection,
//   * the row pass over O: dO_b w for the other half of the residual,
//   * the centred, rounded and packed Gram operand.
// All reductions run in a fixed order, so results are bit-reproducible.
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

// ---------------------------------------------------------------------------
__global__ void k_bind(BindArgs a, int nprob, ProbPtrs* dst) {
  int t = threadIdx.x;
  if (t < nprob) dst[t] = a.p[t];
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// ---------------------------------------------------------------------------
// dE = E - mean(E) per problem, and sum(dE) (needed to make the force exactly
// the centred product).  One workgroup per problem, fixed-order tree sums.
__global__ void __launch_bounds__(256) k_eloc(const ProbDev* probs, const ProbPtrs* ptrs, char* ws) {
  __shared__ double2 red[256];
  const int p = blockIdx.x, t = threadIdx.x;
  const ProbDev P = probs[p];
  const double2* e = ptrs[p].e_loc;
  double2* dE = ws_at<double2>(ws, P.dE_off);
  double2 s = make_double2(0.0, 0.0);
  for (int64_t i = t; i < P.n_s; i += 256) s = cadd(s, e[i]);
  red[t] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) red[t] = cadd(red[t], red[t + w]);
    __syncthreads();
  }
  const double2 mean = cscale(red[0], P.inv_ns);
  __syncthreads();
  s = make_double2(0.0, 0.0);
  for (int64_t i = t; i < P.n_s; i += 256) {
    double2 d = csub(e[i], mean);
    dE[i] = d;
    s = cadd(s, d);
  }
  red[t] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) red[t] = cadd(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) ws_at<double2>(ws, P.scal_off)[0] = red[0];
}

// ---------------------------------------------------------------------------
// Column pass.  Workgroup = one tile of <= 64 columns of one block x one chunk
// of rows; each of the 4 waves reads every 4th row of the chunk, one column per
// lane (a wave reads 64 consecutive elements of a row: coalesced).
//   COL_FORCE   : s1 = sum_x O[x,k],  s2 = sum_x conj(O[x,k]) dE[x]
//   COL_APPLY / COL_BACKPROJ :
//                 s2 = sum_x conj(O[x,k] - mu_k) src_b[x], src_b = u_b
//                 (parameter form), the search direction p_b (sample form,
//                 COL_APPLY) or the solution z_b (sample form, COL_BACKPROJ)
// Partials per (tile, row chunk, lane) are reduced in order by k_colreduce.
constexpr int kColRows = 1024;
template <int DT, int PHASE>
__global__ void __launch_bounds__(256) k_colpass(const ColTile* tiles, const BlockDev* blocks, const ProbDev* probs,
                                                 const ProbPtrs* ptrs, char* ws, double2* part) {
  __shared__ double2 red[2][4][64];
  __shared__ double red3[4][64];
  __shared__ dv2 srcs[kColRows];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const ColTile tile = tiles[blockIdx.x];
  const BlockDev B = blocks[tile.g];
  const ProbDev P = probs[B.prob];
  const ProbPtrs pp = ptrs[B.prob];
  const int RC = gridDim.y, rc = blockIdx.y;
  if (rc >= P.rc) return;
  if (PHASE == COL_APPLY && cg_done(B, ws)) return;
  const int64_t rpc = (P.n_s + P.rc - 1) / P.rc;
  const int64_t r0 = (int64_t)rc * rpc;
  const int64_t r1 = min(P.n_s, r0 + rpc);
  const bool valid = lane < tile.nc;
  const int64_t k = B.col_off + tile.c0 + (valid ? lane : 0);
  const double2* src;
  if (PHASE == COL_FORCE) src = ws_at<double2>(ws, P.dE_off);
  else if (B.form == FORM_P) src = ws_at<double2>(ws, B.u_off);
  else src = ws_at<double2>(ws, PHASE == COL_APPLY ? B.p_off : B.x_off);
  double2 mu = make_double2(0.0, 0.0);
  if (PHASE != COL_FORCE) mu = ws_at<double2>(ws, P.mu_off)[k];
  dv2 s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
  double s3 = 0.0;
  const QGT_GLOBAL dv2* srcv = (const QGT_GLOBAL dv2*)src;
  const dv2 muv = to_dv2(mu);
  const int64_t ldo = pp.ldo;
  // The sample vector is the same for every column: it is staged in LDS, up
  // to kColRows rows at a time, and read from there as a broadcast, which
  // leaves the wave's memory instructions to the rows of O.  Each wave still
  // visits its rows (r0 + w + 4j) in increasing order.
  for (int64_t b0 = r0; b0 < r1; b0 += kColRows) {
    const int64_t b1 = min(r1, b0 + kColRows);
    __syncthreads();  // the previous rows' reads of srcs are done
    for (int64_t i = b0 + t; i < b1; i += 256) srcs[i - b0] = srcv[i];
    __syncthreads();
    if (valid) {
      int64_t r = b0 + w;
      // eight rows in flight per wave
      for (; r + 28 < b1; r += 32) {
        dv2 o[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) o[u] = load_ov<DT>(pp.O, (r + 4 * u) * ldo + k);
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = srcs[r - b0 + 4 * u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (PHASE == COL_FORCE) {
            s1 += o[u];
            s3 = fma(o[u].x, o[u].x, fma(o[u].y, o[u].y, s3));
          } else {
            o[u] -= muv;
          }
          s2 = vfmac(o[u], v[u], s2);
        }
      }
      for (; r < b1; r += 4) {
        dv2 o = load_ov<DT>(pp.O, r * ldo + k);
        if (PHASE == COL_FORCE) {
          s1 += o;
          s3 = fma(o.x, o.x, fma(o.y, o.y, s3));
        } else {
          o -= muv;
        }
        s2 = vfmac(o, srcs[r - b0], s2);
      }
    }
  }
  red[0][w][lane] = to_d2(s1);
  red[1][w][lane] = to_d2(s2);
  red3[w][lane] = s3;
  __syncthreads();
  if (w == 0) {
    double2 a = red[0][0][lane], b = red[1][0][lane];
    double c3 = red3[0][lane];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      a = cadd(a, red[0][q][lane]);
      b = cadd(b, red[1][q][lane]);
      c3 += red3[q][lane];
    }
    const int64_t base = ((int64_t)blockIdx.x * RC + rc) * 64 + lane;
    if (PHASE == COL_FORCE) {
      part[3 * base] = a;
      part[3 * base + 1] = b;
      part[3 * base + 2] = make_double2(c3, 0.0);
    } else {
      part[base] = b;
    }
  }
}

// Ordered reduction of the column-pass partials and the phase epilogue:
//   COL_FORCE   : mu_k = s1 / n_s,  F_k = (s2 - conj(mu_k) sum(dE)) / n_s
//   COL_APPLY  : parameter form r_k = F_k - s2 / n_s - lambda x_k (residual
//                 of (S_b + lambda I) x = F_b); sample form v_k = s2
//   COL_BACKPROJ: delta_k = s2 / n_s (delta_b = dO_b^H z_b / n_s)
template <int PHASE>
__global__ void __launch_bounds__(64) k_colreduce(const ColTile* tiles, const BlockDev* blocks, const ProbDev* probs,
                                                  const ProbPtrs* ptrs, char* ws, const double2* part, int RC) {
  const int lane = threadIdx.x;
  const ColTile tile = tiles[blockIdx.x];
  if (lane >= tile.nc) return;
  const BlockDev B = blocks[tile.g];
  if (PHASE == COL_APPLY && cg_done(B, ws)) return;
  const ProbDev P = probs[B.prob];
  const int64_t c = tile.c0 + lane;  // column within the block
  const int64_t k = B.col_off + c;   // column within the problem
  double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
  double s3 = 0.0;
  for (int rc = 0; rc < P.rc; ++rc) {
    const int64_t base = ((int64_t)blockIdx.x * RC + rc) * 64 + lane;
    if (PHASE == COL_FORCE) {
      s1 = cadd(s1, part[3 * base]);
      s2 = cadd(s2, part[3 * base + 1]);
      s3 += part[3 * base + 2].x;
    } else {
      s2 = cadd(s2, part[base]);
    }
  }
  if (PHASE == COL_FORCE) {
    const double2 mu = cscale(s1, P.inv_ns);
    const double2 sdE = ws_at<double2>(ws, P.scal_off)[0];
    ws_at<double2>(ws, P.mu_off)[k] = mu;
    ws_at<double2>(ws, P.F_off)[k] = cscale(csub(s2, cmulc(mu, sdE)), P.inv_ns);
    ws_at<double>(ws, P.sd_off)[k] = s3 * P.inv_ns - (mu.x * mu.x + mu.y * mu.y);
  } else if (PHASE == COL_APPLY) {
    if (B.form == FORM_P) {
      // q = (S_b + lambda I) p = dO^H (dO p) / n_s + lambda p
      const double2 pv = ws_at<double2>(ws, B.p_off)[c];
      ws_at<double2>(ws, B.q_off)[c] =
          make_double2(fma(s2.x, P.inv_ns, B.lambda * pv.x), fma(s2.y, P.inv_ns, B.lambda * pv.y));
    } else {
      ws_at<double2>(ws, P.v_off)[k] = s2;
    }
  } else {
    ptrs[B.prob].delta[k] = cscale(s2, P.inv_ns);
  }
}

// c_b = sum_{k in b} mu_k w_k: the centring correction of the row pass, so that
// sum_k (O[x,k] - mu_k) w_k = sum_k O[x,k] w_k - c_b.  w = p_b (parameter
// form) or v_b (sample form).  One workgroup per listed block.
// One workgroup of kRedThreads per block; each thread keeps four independent
// partial sums (four loads in flight instead of one dependent chain: the
// pass was latency-bound, 0.26 ms for a 160 400-column block), combined in a
// fixed order, then a fixed-order tree over the workgroup.
constexpr int kRedThreads = 1024;

__global__ void __launch_bounds__(kRedThreads) k_mudot(const int32_t* glist, const BlockDev* blocks,
                                                       const ProbDev* probs, char* ws, double2* bscal) {
  __shared__ double2 red[kRedThreads];
  const int t = threadIdx.x;
  const int g = glist[blockIdx.x];
  const BlockDev B = blocks[g];
  if (cg_done(B, ws)) return;
  const ProbDev P = probs[B.prob];
  const double2* mu = ws_at<double2>(ws, P.mu_off) + B.col_off;
  const double2* wv = B.form == FORM_P ? ws_at<double2>(ws, B.p_off) : ws_at<double2>(ws, P.v_off) + B.col_off;
  double2 s[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  int64_t c = t;
  for (; c + 3 * kRedThreads < B.n_b; c += 4 * kRedThreads) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] = cfma(mu[c + u * kRedThreads], wv[c + u * kRedThreads], s[u]);
  }
  for (; c < B.n_b; c += kRedThreads) s[0] = cfma(mu[c], wv[c], s[0]);
  red[t] = cadd(cadd(s[0], s[1]), cadd(s[2], s[3]));
  __syncthreads();
  for (int q = kRedThreads / 2; q >= 1; q >>= 1) {
    if (t < q) red[t] = cadd(red[t], red[t + q]);
    __syncthreads();
  }
  if (t == 0) bscal[g] = red[0];
}

// Trace of each block QGT, t_b = sum_{k in b} S_kk (a scale estimate of the
// block; S_kk = sum_x |O[x,k]|^2 / n_s - |mu_k|^2 from the column pass).  One
// workgroup per block, fixed-order tree sum.
__global__ void __launch_bounds__(kRedThreads) k_block_trace(const BlockDev* blocks, const ProbDev* probs, char* ws,
                                                             double* trace) {
  __shared__ double red[kRedThreads];
  const int t = threadIdx.x;
  const BlockDev B = blocks[blockIdx.x];
  const double* sd = ws_at<double>(ws, probs[B.prob].sd_off) + B.col_off;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t c = t;
  for (; c + 3 * kRedThreads < B.n_b; c += 4 * kRedThreads) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += sd[c + u * kRedThreads];
  }
  for (; c < B.n_b; c += kRedThreads) s[0] += sd[c];
  red[t] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  for (int q = kRedThreads / 2; q >= 1; q >>= 1) {
    if (t < q) red[t] += red[t + q];
    __syncthreads();
  }
  if (t == 0) trace[blockIdx.x] = red[0];
}

// Row pass.  Workgroup = 16 rows of one block; each wave owns 4 rows and its
// lanes stride over the block's columns (coalesced along the row); the four
// row sums are reduced across the wave with lane shuffles.
//   ROW_P_U     : u_b[x] = sum_k dO[x,k] p_k          (p = search direction)
//   ROW_S_APPLY : q[x] = (sum_k dO[x,k] v_k)/n_s + lambda p[x], v = dO^H p:
//                 q = (T_b + lambda I) p in sample space
template <int DT, int PHASE>
__global__ void __launch_bounds__(256) k_rowpass(const RowItem* items, const BlockDev* blocks, const ProbDev* probs,
                                                 const ProbPtrs* ptrs, char* ws, const double2* bscal) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const RowItem it = items[blockIdx.x];
  const BlockDev B = blocks[it.g];
  if (cg_done(B, ws)) return;
  const ProbDev P = probs[B.prob];
  const ProbPtrs pp = ptrs[B.prob];
  const QGT_GLOBAL dv2* wv = (const QGT_GLOBAL dv2*)(PHASE == ROW_P_U ? ws_at<double2>(ws, B.p_off)
                                                                     : ws_at<double2>(ws, P.v_off) + B.col_off);
  const int64_t rbase = (int64_t)it.r0 + 4 * w;
  // rows past the end are read from the last row (always in bounds) and dropped
  int64_t roff[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) roff[q] = min<int64_t>(rbase + q, P.n_s - 1) * pp.ldo + B.col_off;
  dv2 acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  int64_t c = lane;
  // two column chunks (eight loads of O) in flight per lane
  for (; c + 64 < B.n_b; c += 128) {
    const dv2 w0 = wv[c], w1 = wv[c + 64];
    dv2 o0[4], o1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      o0[q] = load_ov<DT>(pp.O, roff[q] + c);
      o1[q] = load_ov<DT>(pp.O, roff[q] + c + 64);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = vfma(o1[q], w1, vfma(o0[q], w0, acc[q]));
  }
  if (c < B.n_b) {
    const dv2 w0 = wv[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = vfma(load_ov<DT>(pp.O, roff[q] + c), w0, acc[q]);
  }
  const double2 cb = bscal[it.g];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double re = wave_sum(acc[q].x), im = wave_sum(acc[q].y);
    if (lane == q && rbase + q < P.n_s) {
      const int64_t x = rbase + q;
      const double2 tsum = make_double2(re - cb.x, im - cb.y);
      if (PHASE == ROW_P_U) {
        ws_at<double2>(ws, B.u_off)[x] = tsum;
      } else {
        const double2 pv = ws_at<double2>(ws, B.p_off)[x];
        ws_at<double2>(ws, B.q_off)[x] =
            make_double2(fma(tsum.x, P.inv_ns, B.lambda * pv.x), fma(tsum.y, P.inv_ns, B.lambda * pv.y));
      }
    }
  }
}

// One k-group of the packed operand (16 bytes, 16-byte aligned) as a single
// vector store rather than G element stores.
template <typename T, int G>
__device__ __forceinline__ void store_group16(T* dst, const T (&v)[G]) {
  static_assert(sizeof(T) * G == 16, "a k-group is 16 bytes");
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  u4v u;
  __builtin_memcpy(&u, v, 16);
  *(QGT_GLOBAL u4v*)dst = u;
}

// ---------------------------------------------------------------------------
// Centre and pack the Gram operand of one block.  The packed operand P (K_pad x
// m_pad, planar Re and Im) is laid out with the contraction index k in groups of
// G: element (k, m) sits at ((k / G) * m_pad + m) * G + k % G.  Padding is zero.
//   parameter form: P[k][m] = O[k, off + m] - mu      (k = sample, m = parameter)
//   sample form   : P[k][m] = conj(O[m, off + k] - mu) (k = parameter, m = sample)
// so that in both cases the Gram is G[i][j] = sum_k conj(P[k][i]) P[k][j].
// The centred value is formed in FP64 and rounded once.
template <int DT, int PREC>
__global__ void __launch_bounds__(256) k_pack(const int32_t* glist, const BlockDev* blocks, const ProbDev* probs,
                                              const ProbPtrs* ptrs, char* ws, int form) {
  typedef typename PackT<PREC>::T T;
  constexpr int G = pack_group(PREC);
  const int t = threadIdx.x;
  const int g = glist[blockIdx.z];
  const BlockDev B = blocks[g];
  if (B.form != form) return;
  const int64_t mtile = (int64_t)blockIdx.x * 64 * (form == FORM_P ? 1 : kPackRowsS);
  if (mtile >= B.m_pad) return;
  const ProbDev P = probs[B.prob];
  const ProbPtrs pp = ptrs[B.prob];
  const double2* mu = ws_at<double2>(ws, P.mu_off) + B.col_off;
  T* re = ws_at<T>(ws, B.pack_off);
  T* im = re + B.K_pad * B.m_pad;
  const int64_t ngroups = B.K_pad / G;
  if (form == FORM_P) {
    // lanes along m (columns of O): each row read is coalesced
    const int64_t m = mtile + (t & 63);
    const bool mvalid = m < B.n_b;
    const int64_t mc = mvalid ? m : B.n_b - 1;  // in-bounds column for the loads
    const dv2 mum = to_dv2(mu[mc]);
    for (int64_t kg = (int64_t)blockIdx.y * 4 + (t >> 6); kg < ngroups; kg += (int64_t)gridDim.y * 4) {
      T vr[G], vi[G];
      dv2 o[G];
#pragma unroll
      for (int e = 0; e < G; ++e) o[e] = load_ov<DT>(pp.O, min<int64_t>(kg * G + e, P.n_s - 1) * pp.ldo + B.col_off + mc);
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const bool ok = mvalid && kg * G + e < P.n_s;
        const dv2 v = ok ? o[e] - mum : dv2{0.0, 0.0};
        vr[e] = to_pack<PREC>(v.x);
        vi[e] = to_pack<PREC>(v.y);
      }
      const int64_t dst = (kg * B.m_pad + m) * G;
      store_group16(re + dst, vr);
      store_group16(im + dst, vi);
    }
  } else {
    // 4 lanes cover 4 consecutive k-groups of one row of O (contiguous reads),
    // 16 rows per wave.  Each thread keeps one k-group, and with it the G
    // column means, for 64 * kPackRowsS rows of the block (ngroups is a
    // multiple of 4, so every lane of a workgroup has a valid k-group).
    const int kq = t & 3;
    const int64_t m_end = min<int64_t>(mtile + 64 * kPackRowsS, B.m_pad);
    for (int64_t kg = (int64_t)blockIdx.y * 4 + kq; kg < ngroups; kg += (int64_t)gridDim.y * 4) {
      const bool whole = kg * G + G <= B.n_b;
      dv2 mk[G];
#pragma unroll
      for (int e = 0; e < G; ++e) mk[e] = to_dv2(mu[min<int64_t>(kg * G + e, B.n_b - 1)]);
      for (int64_t m = mtile + (t >> 2); m < m_end; m += 64) {
        const bool mvalid = m < P.n_s;
        const int64_t rowoff = (mvalid ? m : P.n_s - 1) * pp.ldo + B.col_off;  // in-bounds row for the loads
        T vr[G], vi[G];
        dv2 o[G];
        if (DT == 0 && G >= 2 && whole && ((rowoff + kg * G) & 1) == 0) {
          // the whole group is inside the block and 16-byte aligned: two
          // complex64 values per load
          const QGT_GLOBAL f4v* p4 = (const QGT_GLOBAL f4v*)((const QGT_GLOBAL fv2*)pp.O + rowoff + kg * G);
#pragma unroll
          for (int h = 0; h < G / 2; ++h) {
            const f4v f = p4[h];
            o[2 * h] = dv2{(double)f.x, (double)f.y};
            o[2 * h + 1] = dv2{(double)f.z, (double)f.w};
          }
        } else {
#pragma unroll
          for (int e = 0; e < G; ++e) o[e] = load_ov<DT>(pp.O, rowoff + min<int64_t>(kg * G + e, B.n_b - 1));
        }
#pragma unroll
        for (int e = 0; e < G; ++e) {
          const bool ok = mvalid && kg * G + e < B.n_b;
          const dv2 v = ok ? o[e] - mk[e] : dv2{0.0, 0.0};
          vr[e] = to_pack<PREC>(v.x);
          vi[e] = to_pack<PREC>(-v.y);
        }
        const int64_t dst = (kg * B.m_pad + m) * G;
        store_group16(re + dst, vr);
        store_group16(im + dst, vi);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Preconditioned conjugate gradients, in FP64, on the shifted block system
// (S_b + lambda I) x = F_b (parameter form) or (T_b + lambda I) z = dE (sample
// form).  The operator A is applied matrix-free from O by the column and row
// passes; the preconditioner M = L L^H is the Cholesky factor of the shifted
// Gram, which may have been accumulated in a lower precision.  The iterate
// therefore converges to the FP64 solution whatever the Gram precision, and a
// few eigenvalues of M^{-1} A far from one (directions the rounded Gram gets
// wrong) cost a few iterations rather than stalling the iteration.
//   CG_START : rho = r^H z, p = z            (x = 0, r = rhs, z = M^{-1} r)
//   CG_ALPHA : alpha = rho / p^H q, x += alpha p, r -= alpha q   (q = A p)
//   CG_BETA  : rho' = r^H z, p = z + (rho' / rho) p, rho = rho'
//              and the convergence test: est = ||z|| / ||x + z||, the size of
//              the preconditioned correction relative to the corrected
//              solution; a block with est <= rtol (rtol > 0) is done: every
//              later pass skips it and its z is kept for CG_FINAL
//   CG_FINAL : x += z (one more preconditioned correction with the last
//              residual) and est as above for blocks still running; status
//              QGT_ERR_NOT_CONVERGED when rtol > 0, at least one iteration ran
//              and est > rtol.
// The test uses the correction itself rather than a predicted error after it
// (correction times the observed contraction of successive corrections): the
// first CG step removes the bulk of the error, and directions the
// preconditioner damps (the null vector 1 of a sample-form block, shifted up by
// the rank-one term) hide error from z for a step or two, so the contraction
// of the early corrections can promise far more than the next step delivers.
// One workgroup per block; fixed-order tree reductions (bit-reproducible).
// Entries at and beyond m are padding: they are neither read nor written here.
template <int PHASE>
__global__ void __launch_bounds__(kRedThreads) k_cg(const BlockDev* blocks, char* ws, CgScal* cg, double rtol,
                                                    int iters, int32_t* status) {
  __shared__ double red[3][kRedThreads];
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const BlockDev B = blocks[g];
  const int64_t m = B.m;
  double2* x = ws_at<double2>(ws, B.x_off);
  double2* r = ws_at<double2>(ws, B.r_off);
  const double2* z = ws_at<double2>(ws, B.z_off);
  double2* p = ws_at<double2>(ws, B.p_off);
  const double2* q = ws_at<double2>(ws, B.q_off);
  const double rho = cg[g].rho;
  const bool done = cg[g].done != 0;
  if ((PHASE == CG_ALPHA || PHASE == CG_BETA) && done) return;
  double a = 0.0, b = 0.0, xx = 0.0;
  for (int64_t i = t; i < m; i += kRedThreads) {
    if (PHASE == CG_START || PHASE == CG_BETA) {
      const double2 ri = r[i], zi = z[i];
      a = fma(ri.x, zi.x, fma(ri.y, zi.y, a));
      b = fma(zi.x, zi.x, fma(zi.y, zi.y, b));
      if (PHASE == CG_BETA) {
        const double2 xn = cadd(x[i], zi);
        xx = fma(xn.x, xn.x, fma(xn.y, xn.y, xx));
      }
    } else if (PHASE == CG_ALPHA) {
      const double2 pi = p[i], qi = q[i];
      a = fma(pi.x, qi.x, fma(pi.y, qi.y, a));
    } else {
      const double2 zi = z[i];
      const double2 xn = cadd(x[i], zi);
      x[i] = xn;
      a = fma(zi.x, zi.x, fma(zi.y, zi.y, a));
      b = fma(xn.x, xn.x, fma(xn.y, xn.y, b));
    }
  }
  red[0][t] = a;
  red[1][t] = b;
  red[2][t] = xx;
  __syncthreads();
  for (int h = kRedThreads / 2; h >= 1; h >>= 1) {
    if (t < h) {
      red[0][t] += red[0][t + h];
      red[1][t] += red[1][t + h];
      red[2][t] += red[2][t + h];
    }
    __syncthreads();
  }
  a = red[0][0];
  b = red[1][0];
  xx = red[2][0];
  if (PHASE == CG_START) {
    for (int64_t i = t; i < m; i += kRedThreads) p[i] = z[i];
    if (t == 0) cg[g].rho = a;
  } else if (PHASE == CG_ALPHA) {
    // p^H A p > 0 for the Hermitian positive definite A unless p = 0
    const double alpha = (a > 0.0 && a < INFINITY) ? rho / a : 0.0;
    for (int64_t i = t; i < m; i += kRedThreads) {
      const double2 pi = p[i], qi = q[i], xi = x[i], ri = r[i];
      x[i] = make_double2(fma(alpha, pi.x, xi.x), fma(alpha, pi.y, xi.y));
      r[i] = make_double2(fma(-alpha, qi.x, ri.x), fma(-alpha, qi.y, ri.y));
    }
    if (t == 0) cg[g].iters += 1;
  } else if (PHASE == CG_BETA) {
    // convergence test on this iteration's correction z; a block that meets
    // rtol stops here (z is kept for the final step)
    const double est = xx > 0.0 ? sqrt(b / xx) : (b > 0.0 ? INFINITY : 0.0);
    const bool conv = rtol > 0.0 && est <= rtol;
    if (!conv) {
      const double beta = rho > 0.0 ? a / rho : 0.0;
      for (int64_t i = t; i < m; i += kRedThreads) {
        const double2 pi = p[i], zi = z[i];
        p[i] = make_double2(fma(beta, pi.x, zi.x), fma(beta, pi.y, zi.y));
      }
    }
    if (t == 0) {
      cg[g].rho = a;
      if (conv) {
        cg[g].est = est;
        cg[g].done = 1;
      }
    }
  } else {
    if (t == 0 && !done) cg[g].est = b > 0.0 ? sqrt(a / b) : (a > 0.0 ? INFINITY : 0.0);
    if (t == 0 && rtol > 0.0 && iters > 0 && !(cg[g].est <= rtol) && status[g] == 0)
      status[g] = 6;  // QGT_ERR_NOT_CONVERGED
  }
}

// ---------------------------------------------------------------------------
// Solve set-up: x = 0 and r = right-hand side (F_b for the parameter form, dE
// for the sample form), zero padding to m_pad.
__global__ void __launch_bounds__(256) k_init_solve(const BlockDev* blocks, const ProbDev* probs, char* ws) {
  const BlockDev B = blocks[blockIdx.y];
  const ProbDev P = probs[B.prob];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {
    CgScal* cg = reinterpret_cast<CgScal*>(ws + B.cg_off);
    cg->done = 0;
    cg->iters = 0;
  }
  if (i >= B.m_pad) return;
  double2 rhs = make_double2(0.0, 0.0);
  if (i < B.m) rhs = B.form == FORM_P ? ws_at<double2>(ws, P.F_off)[B.col_off + i] : ws_at<double2>(ws, P.dE_off)[i];
  ws_at<double2>(ws, B.r_off)[i] = rhs;
  ws_at<double2>(ws, B.x_off)[i] = make_double2(0.0, 0.0);
}

// delta[off + i] = x_b[i] for parameter-form blocks.
__global__ void __launch_bounds__(256) k_scatter_p(const BlockDev* blocks, const ProbPtrs* ptrs, char* ws) {
  const BlockDev B = blocks[blockIdx.y];
  if (B.form != FORM_P) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= B.n_b) return;
  ptrs[B.prob].delta[B.col_off + i] = ws_at<double2>(ws, B.x_off)[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_bind(const BindArgs& a, int nprob, ProbPtrs* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_bind, dim3(1), dim3(kMaxProblems), 0, s, a, nprob, dst);
}

void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

void launch_eloc(const ProbDev* probs, const ProbPtrs* ptrs, char* ws, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_eloc, dim3(nprob), dim3(256), 0, s, probs, ptrs, ws);
}

template <int DT>
static void colpass_dt(int phase, const ColTile* tiles, int ntiles, int RC, const BlockDev* blocks,
                       const ProbDev* probs, const ProbPtrs* ptrs, char* ws, double2* part, hipStream_t s) {
  dim3 grid(ntiles, RC);
  if (phase == COL_FORCE)
    hipLaunchKernelGGL((k_colpass<DT, COL_FORCE>), grid, dim3(256), 0, s, tiles, blocks, probs, ptrs, ws, part);
  else if (phase == COL_APPLY)
    hipLaunchKernelGGL((k_colpass<DT, COL_APPLY>), grid, dim3(256), 0, s, tiles, blocks, probs, ptrs, ws, part);
  else
    hipLaunchKernelGGL((k_colpass<DT, COL_BACKPROJ>), grid, dim3(256), 0, s, tiles, blocks, probs, ptrs, ws, part);
}

void launch_colpass(int dt, int phase, const ColTile* tiles, int ntiles, int RC, const BlockDev* blocks,
                    const ProbDev* probs, const ProbPtrs* ptrs, char* ws, double2* part, hipStream_t s) {
  if (ntiles <= 0) return;
  if (dt == 0) colpass_dt<0>(phase, tiles, ntiles, RC, blocks, probs, ptrs, ws, part, s);
  else colpass_dt<1>(phase, tiles, ntiles, RC, blocks, probs, ptrs, ws, part, s);
  dim3 grid(ntiles);
  if (phase == COL_FORCE)
    hipLaunchKernelGGL((k_colreduce<COL_FORCE>), grid, dim3(64), 0, s, tiles, blocks, probs, ptrs, ws, part, RC);
  else if (phase == COL_APPLY)
    hipLaunchKernelGGL((k_colreduce<COL_APPLY>), grid, dim3(64), 0, s, tiles, blocks, probs, ptrs, ws, part, RC);
  else
    hipLaunchKernelGGL((k_colreduce<COL_BACKPROJ>), grid, dim3(64), 0, s, tiles, blocks, probs, ptrs, ws, part, RC);
}

void launch_block_trace(const BlockDev* blocks, const ProbDev* probs, char* ws, double* trace, int nblocks,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_block_trace, dim3(nblocks), dim3(kRedThreads), 0, s, blocks, probs, ws, trace);
}

void launch_mudot(const int32_t* glist, int n, const BlockDev* blocks, const ProbDev* probs, char* ws,
                  double2* bscal, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mudot, dim3(n), dim3(kRedThreads), 0, s, glist, blocks, probs, ws, bscal);
}

void launch_rowpass(int dt, int phase, const RowItem* items, int nitems, const BlockDev* blocks,
                    const ProbDev* probs, const ProbPtrs* ptrs, char* ws, const double2* bscal, hipStream_t s) {
  if (nitems <= 0) return;
  dim3 grid(nitems);
  if (dt == 0) {
    if (phase == ROW_P_U) hipLaunchKernelGGL((k_rowpass<0, ROW_P_U>), grid, dim3(256), 0, s, items, blocks, probs, ptrs, ws, bscal);
    else hipLaunchKernelGGL((k_rowpass<0, ROW_S_APPLY>), grid, dim3(256), 0, s, items, blocks, probs, ptrs, ws, bscal);
  } else {
    if (phase == ROW_P_U) hipLaunchKernelGGL((k_rowpass<1, ROW_P_U>), grid, dim3(256), 0, s, items, blocks, probs, ptrs, ws, bscal);
    else hipLaunchKernelGGL((k_rowpass<1, ROW_S_APPLY>), grid, dim3(256), 0, s, items, blocks, probs, ptrs, ws, bscal);
  }
}

template <int DT, int PREC>
static void pack_launch(const int32_t* glist, int n, int64_t max_mtiles, int ygrid, const BlockDev* blocks,
                        const ProbDev* probs, const ProbPtrs* ptrs, char* ws, int form, hipStream_t s) {
  dim3 grid((unsigned)max_mtiles, ygrid, n);
  hipLaunchKernelGGL((k_pack<DT, PREC>), grid, dim3(256), 0, s, glist, blocks, probs, ptrs, ws, form);
}

void launch_pack(int dt, int prec, const int32_t* glist, int n, int64_t max_mtiles, int ygrid, const BlockDev* blocks,
                 const ProbDev* probs, const ProbPtrs* ptrs, char* ws, int form, hipStream_t s) {
  if (n <= 0) return;
  if (dt == 0) {
    if (prec == PREC_FP64) pack_launch<0, PREC_FP64>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
    else if (prec == PREC_FP32) pack_launch<0, PREC_FP32>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
    else pack_launch<0, PREC_BF16>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
  } else {
    if (prec == PREC_FP64) pack_launch<1, PREC_FP64>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
    else if (prec == PREC_FP32) pack_launch<1, PREC_FP32>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
    else pack_launch<1, PREC_BF16>(glist, n, max_mtiles, ygrid, blocks, probs, ptrs, ws, form, s);
  }
}

void launch_cg(int phase, const BlockDev* blocks, char* ws, CgScal* cg, double rtol, int iters, int32_t* status,
               int nblocks, hipStream_t s) {
  const dim3 grid(nblocks), blk(kRedThreads);
  if (phase == CG_START) hipLaunchKernelGGL(k_cg<CG_START>, grid, blk, 0, s, blocks, ws, cg, rtol, iters, status);
  else if (phase == CG_ALPHA) hipLaunchKernelGGL(k_cg<CG_ALPHA>, grid, blk, 0, s, blocks, ws, cg, rtol, iters, status);
  else if (phase == CG_BETA) hipLaunchKernelGGL(k_cg<CG_BETA>, grid, blk, 0, s, blocks, ws, cg, rtol, iters, status);
  else hipLaunchKernelGGL(k_cg<CG_FINAL>, grid, blk, 0, s, blocks, ws, cg, rtol, iters, status);
}

void launch_init_solve(const BlockDev* blocks, const ProbDev* probs, char* ws, int nblocks, int64_t max_mpad,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_init_solve, dim3((unsigned)((max_mpad + 255) / 256), nblocks), dim3(256), 0, s, blocks, probs, ws);
}

void launch_scatter_p(const BlockDev* blocks, const ProbPtrs* ptrs, char* ws, int nblocks, int64_t max_nb,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_p, dim3((unsigned)((max_nb + 255) / 256), nblocks), dim3(256), 0, s, blocks, ptrs, ws);
}

}  // namespace qgt
