// Complex Hermitian block Gram on the gfx950 matrix cores.
//
// For each block, G = P^H P over the packed operand P (K x m, planar Re/Im), so
// that Re G = R^T R + I^T I and Im G = R^T I - I^T R (the four real products of
// the real/imaginary split).  The parameter form gives n_s * S_b (Eq. 2 and
// Eq. 3), the sample form n_s * T_b.  Only lower-triangle 64x64 output tiles
// are computed.  The epilogue scales by 1/n_s, adds the uniform shift lambda on
// the diagonal (Sec. 2) and writes FP64 complex; padding rows and columns get a
// unit diagonal so that the padded matrix stays positive definite.
//
// Workgroup: 256 threads = 4 waves in a 2x2 arrangement, each wave a 32x32
// output sub-tile (2x2 MFMA 16x16 tiles, Re and Im accumulators).  The
// contraction runs in LDS stages (double-buffered through registers); the
// packed layout lets every lane fetch its MFMA inputs for one k-group with one
// contiguous LDS read.
//   FP64: v_mfma_f64_16x16x4_f64, 4 k per group
//   FP32: v_mfma_f32_16x16x4_f32, 4 k per group
//   BF16: v_mfma_f32_16x16x32_bf16 (FP32 accumulation), 8 k per group
// Work items are spread over the 8 XCDs in contiguous chunks of similar cost so
// that tiles sharing operand panels run under the same L2.
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

template <int PREC>
struct GramCfg {
  static constexpr int G = pack_group(PREC);
  static constexpr int KS = gram_stage_k(PREC);
  static constexpr int SG = KS / G;             // k-groups per stage
  static constexpr int RUN = 64 * G;            // elements of one group run of a 64-column tile
  static constexpr int PANEL = SG * RUN;        // elements per panel per stage
  static constexpr int ESZ = prec_bytes(PREC);
  static constexpr int CPR = RUN * ESZ / 16;    // 16-byte chunks per run
  static constexpr int CPP = SG * CPR;          // 16-byte chunks per panel
  static constexpr int CPT = 4 * CPP / 256;     // chunks per thread per stage
};

template <int PREC>
__device__ __forceinline__ void gram_load_stage(uint4 (&reg)[GramCfg<PREC>::CPT], const char* re_base,
                                                const char* im_base, int64_t m_pad, int ti, int tj, int st) {
  typedef GramCfg<PREC> C;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < C::CPT; ++j) {
    const int c = t + 256 * j;
    const int panel = c / C::CPP;
    const int q = c % C::CPP;
    const int run = q / C::CPR;
    const int off = q % C::CPR;
    const char* plane = (panel & 1) ? im_base : re_base;
    const int tile = (panel < 2) ? ti : tj;
    const int64_t grp = (int64_t)st * C::SG + run;
    const int64_t elem = (grp * m_pad + (int64_t)tile * 64) * C::G;
    reg[j] = *reinterpret_cast<const uint4*>(plane + elem * C::ESZ + (int64_t)off * 16);
  }
}

template <int PREC>
__device__ __forceinline__ void gram_store_stage(const uint4 (&reg)[GramCfg<PREC>::CPT], char* lds_buf) {
  typedef GramCfg<PREC> C;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < C::CPT; ++j) {
    const int c = t + 256 * j;
    reinterpret_cast<uint4*>(lds_buf)[c] = reg[j];
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_gram(const GramItem* items, XcdChunks chunks, const BlockDev* blocks,
                                              char* ws, double2* part) {
  typedef GramCfg<PREC> C;
  typedef typename PackT<PREC>::T T;
  __shared__ __attribute__((aligned(16))) char lds[2][4 * C::PANEL * C::ESZ];

  // XCD-aware mapping: workgroup w runs on XCD w % 8 and takes the next item of
  // that XCD's chunk.
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  if (jx >= chunks.len[x]) return;
  const GramItem it = items[chunks.start[x] + jx];
  const BlockDev B = blocks[it.g];
  const char* re_base = ws + B.pack_off;
  const char* im_base = re_base + B.K_pad * B.m_pad * C::ESZ;

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l16 = lane & 15, lg = lane >> 4;

  typedef typename std::conditional<PREC == PREC_FP64, d4v, f4v>::type acc_t;
  acc_t accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }

  uint4 reg[C::CPT];
  gram_load_stage<PREC>(reg, re_base, im_base, B.m_pad, it.ti, it.tj, it.s0);
  gram_store_stage<PREC>(reg, lds[0]);
  __syncthreads();
  int cur = 0;
  for (int st = it.s0; st < it.s1; ++st) {
    const bool more = st + 1 < it.s1;
    if (more) gram_load_stage<PREC>(reg, re_base, im_base, B.m_pad, it.ti, it.tj, st + 1);
    const T* P = reinterpret_cast<const T*>(lds[cur]);
#pragma unroll
    for (int q = 0; q < C::SG / 4; ++q) {
      const int grp = 4 * q + lg;
      if constexpr (PREC == PREC_BF16) {
        bf8v aR[2], aI[2], bR[2], bI[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int ca = 32 * wr + 16 * s + l16, cb = 32 * wc + 16 * s + l16;
          aR[s] = *reinterpret_cast<const bf8v*>(P + 0 * C::PANEL + grp * C::RUN + ca * C::G);
          uint4 ai = *reinterpret_cast<const uint4*>(P + 1 * C::PANEL + grp * C::RUN + ca * C::G);
          ai.x ^= 0x80008000u; ai.y ^= 0x80008000u; ai.z ^= 0x80008000u; ai.w ^= 0x80008000u;  // -I
          aI[s] = *reinterpret_cast<const bf8v*>(&ai);
          bR[s] = *reinterpret_cast<const bf8v*>(P + 2 * C::PANEL + grp * C::RUN + cb * C::G);
          bI[s] = *reinterpret_cast<const bf8v*>(P + 3 * C::PANEL + grp * C::RUN + cb * C::G);
        }
        // aI holds -I: Re += R R^T + (-I)(-I)... use the sign once for each product
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR[a], bR[b], accR[a][b], 0, 0, 0);
            accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR[a], bI[b], accI[a][b], 0, 0, 0);
            accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aI[a], bR[b], accI[a][b], 0, 0, 0);
          }
        // Re needs +I_i^T I_j: negate the B side of the negated A (-I_i)(-I_j)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          uint4 bi = *reinterpret_cast<const uint4*>(&bI[b]);
          bi.x ^= 0x80008000u; bi.y ^= 0x80008000u; bi.z ^= 0x80008000u; bi.w ^= 0x80008000u;
          bI[b] = *reinterpret_cast<const bf8v*>(&bi);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aI[a], bI[b], accR[a][b], 0, 0, 0);
      } else {
        typedef typename std::conditional<PREC == PREC_FP64, d4v, f4v>::type v4;
        v4 aR[2], aI[2], bR[2], bI[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int ca = 32 * wr + 16 * s + l16, cb = 32 * wc + 16 * s + l16;
          aR[s] = *reinterpret_cast<const v4*>(P + 0 * C::PANEL + grp * C::RUN + ca * C::G);
          aI[s] = *reinterpret_cast<const v4*>(P + 1 * C::PANEL + grp * C::RUN + ca * C::G);
          bR[s] = *reinterpret_cast<const v4*>(P + 2 * C::PANEL + grp * C::RUN + cb * C::G);
          bI[s] = *reinterpret_cast<const v4*>(P + 3 * C::PANEL + grp * C::RUN + cb * C::G);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              if constexpr (PREC == PREC_FP64) {
                accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[a][e], bR[b][e], accR[a][b], 0, 0, 0);
                accR[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aI[a][e], bI[b][e], accR[a][b], 0, 0, 0);
                accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aR[a][e], bI[b][e], accI[a][b], 0, 0, 0);
                accI[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aI[a][e], bR[b][e], accI[a][b], 0, 0, 0);
              } else {
                accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aR[a][e], bR[b][e], accR[a][b], 0, 0, 0);
                accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aI[a][e], bI[b][e], accR[a][b], 0, 0, 0);
                accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aR[a][e], bI[b][e], accI[a][b], 0, 0, 0);
                accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-aI[a][e], bR[b][e], accI[a][b], 0, 0, 0);
              }
            }
      }
    }
    if (more) gram_store_stage<PREC>(reg, lds[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
  }

  // Epilogue.  Output layout of the 16x16 MFMA tiles: lane l, register r holds
  // row 4*(l/16)+r (FP32/BF16) or 4*r+l/16 (FP64), column l%16.
  double2* A = ws_at<double2>(ws, B.mat_off);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int iloc = 32 * wr + 16 * a + (PREC == PREC_FP64 ? 4 * r + lg : 4 * lg + r);
        const int jloc = 32 * wc + 16 * b + l16;
        double re = (double)accR[a][b][r], im = (double)accI[a][b][r];
        if (it.slot >= 0) {
          part[((int64_t)it.slot * 64 + iloc) * 64 + jloc] = make_double2(re, im);
        } else {
          const int64_t R = (int64_t)it.ti * 64 + iloc, Cc = (int64_t)it.tj * 64 + jloc;
          re *= B.inv_ns;
          im *= B.inv_ns;
          if (R == Cc) {
            re = R < B.m ? re + B.lambda : 1.0;
            im = 0.0;
          }
          A[R * B.m_pad + Cc] = make_double2(re, im);
        }
      }
}

// Ordered sum of split-K partial tiles, then the same epilogue.
__global__ void __launch_bounds__(256) k_gram_splitk_reduce(const SplitItem* items, const BlockDev* blocks, char* ws,
                                                            const double2* part) {
  const SplitItem it = items[blockIdx.x];
  const BlockDev B = blocks[it.g];
  double2* A = ws_at<double2>(ws, B.mat_off);
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int iloc = idx >> 6, jloc = idx & 63;
    double2 s = part[(int64_t)it.slot0 * 4096 + idx];
    for (int q = 1; q < it.nsplit; ++q) s = cadd(s, part[(int64_t)(it.slot0 + q) * 4096 + idx]);
    const int64_t R = (int64_t)it.ti * 64 + iloc, Cc = (int64_t)it.tj * 64 + jloc;
    double re = s.x * B.inv_ns, im = s.y * B.inv_ns;
    if (R == Cc) {
      re = R < B.m ? re + B.lambda : 1.0;
      im = 0.0;
    }
    A[R * B.m_pad + Cc] = make_double2(re, im);
  }
}

void launch_gram(int prec, const GramItem* items, const XcdChunks& chunks, const BlockDev* blocks, char* ws,
                 double2* part, hipStream_t s) {
  int maxlen = 0;
  for (int i = 0; i < 8; ++i) maxlen = chunks.len[i] > maxlen ? chunks.len[i] : maxlen;
  if (maxlen == 0) return;
  dim3 grid(8 * maxlen);
  if (prec == PREC_FP64) hipLaunchKernelGGL(k_gram<PREC_FP64>, grid, dim3(256), 0, s, items, chunks, blocks, ws, part);
  else if (prec == PREC_FP32) hipLaunchKernelGGL(k_gram<PREC_FP32>, grid, dim3(256), 0, s, items, chunks, blocks, ws, part);
  else hipLaunchKernelGGL(k_gram<PREC_BF16>, grid, dim3(256), 0, s, items, chunks, blocks, ws, part);
}

void launch_gram_splitk_reduce(const SplitItem* items, int n, const BlockDev* blocks, char* ws, const double2* part,
                               hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gram_splitk_reduce, dim3(n), dim3(256), 0, s, items, blocks, ws, part);
}

}  // namespace qgt
