// Complex Hermitian block Gram on the gfx950 matrix cores.
//
// For each block, G = P^H P over the packed operand P (K x m, planar Re/Im), so
// that Re G = R^T R + I^T I and Im G = R^T I - I^T R (the four real products of
// the real/imaginary split).  The parameter form gives n_s * S_b (Eq. 2 and
// Eq. 3), the sample form n_s * T_b.  Only lower-triangle 128x128 output tiles
// are computed.  The epilogue scales by 1/n_s, adds the uniform shift lambda on
// the diagonal (Sec. 2) and writes complex FP64 (or complex FP32 where the plan
// factors the block in FP32); padding rows and columns get a unit diagonal so
// that the padded matrix stays positive definite.
//
// Workgroup: FP32 uses 4 waves in a 2x2 arrangement, each wave a 64x64 output
// sub-tile (4x4 MFMA 16x16 tiles, Re and Im accumulators); FP64 and BF16 use 8
// waves in a 2x4 arrangement of 64x32 sub-tiles (FP64 so that its
// accumulators fit the registers, BF16 so that two waves per SIMD hide each
// other's LDS reads behind their short MFMAs).  Operands
// stream through a ring of three 32 KB LDS stages filled by asynchronous
// global-to-LDS loads (global_load_lds_dwordx4) two stages ahead; one barrier
// per stage.  A stage holds four k-groups of the four operand panels (Re and Im
// of the row tile and of the column tile); every lane reads one 16-byte
// fragment per operand and sub-tile:
//   FP64: v_mfma_f64_16x16x4_f64, k-group of 2
//   FP32: v_mfma_f32_16x16x4_f32, k-group of 4
//   BF16: v_mfma_f32_16x16x32_bf16 (FP32 accumulation), k-group of 8
// Work items are spread over the 8 XCDs (workgroup w runs on XCD w % 8): each
// XCD's list holds an eighth of every block's tiles, contiguous in patch order,
// so that the tiles one XCD runs at a time share operand panels in its L2.
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

constexpr int kStageBytes = 32768;
constexpr int kPanelBytes = 8192;  // 4 k-groups x 128 columns x 16 bytes

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// s_waitcnt vmcnt(n), other counters unconstrained (gfx9 encoding).
#define QGT_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 15) | ((((n) >> 4) & 3) << 14))
// s_waitcnt lgkmcnt(0), other counters unconstrained.
#define QGT_WAIT_LGKMCNT0() __builtin_amdgcn_s_waitcnt(0xC07F)

// -v for eight BF16 values (sign-bit flip on the register value).  Operands
// are read from LDS with their own BF16 vector type and negated in registers:
// an LDS read through an integer type is taken by the compiler as possibly
// aliasing the asynchronous LDS stores of the prefetched stages and makes it
// wait for all of them (vmcnt(0)) before the read, which would serialise the
// operand pipeline.
__device__ __forceinline__ bf8v bf8_neg(bf8v v) {
  uint4 u = __builtin_bit_cast(uint4, v);
  u.x ^= 0x80008000u;
  u.y ^= 0x80008000u;
  u.z ^= 0x80008000u;
  u.w ^= 0x80008000u;
  return __builtin_bit_cast(bf8v, u);
}

template <int PREC>
struct GramShape {
  // FP64 and BF16: 8 waves (two per SIMD) of 64x32 sub-tiles, so that one
  // wave's MFMAs hide the other's LDS reads; FP32, whose MFMAs are longest per
  // byte of operand, keeps 4 waves of 64x64.
  static constexpr int NW = PREC == PREC_FP32 ? 4 : 8;  // waves per workgroup
  static constexpr int SB = PREC == PREC_FP32 ? 4 : 2;  // 16-column sub-tiles per wave
  static constexpr int LPW = 32 / NW;                   // 1 KB loads per wave per stage
};

// The asynchronous global -> LDS loads of one stage: 32 wave instructions of
// 1 KB (64 columns x 16 bytes), spread over the waves.  Each wave's share is
// described once per work item (the lane's source address for the item's
// first stage, the uniform destination offset in a stage buffer), so that
// issuing a stage costs an address increment and the load per slot.  The
// wave index is made provably uniform: the LDS destination is taken from a
// scalar register, so it must not need a per-lane loop.
template <int NW>
struct GramLoads {
  // Fixed-size arrays (NW >= 4): an operand type that depends on NW would make
  // the target builtin below a dependent call, which the host pass of the
  // compiler cannot resolve and then drops the kernel's launch stub.
  const char* src[8];
  int dst[8];

  __device__ __forceinline__ void init(const char* re_base, const char* im_base, int64_t m_pad, int ti, int tj,
                                       int st0) {
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int u = 0; u < 32 / NW; ++u) {
      const int qi = w * (32 / NW) + u;  // 0..31
      const int panel = qi >> 3;         // Re_i, Im_i, Re_j, Im_j
      const int grp = (qi >> 1) & 3;     // k-group within the stage
      const int half = qi & 1;           // columns 0-63 or 64-127 of the tile
      const char* plane = (panel & 1) ? im_base : re_base;
      const int tile = panel < 2 ? ti : tj;
      const int64_t col = (int64_t)tile * 128 + half * 64 + lane;
      src[u] = plane + (((int64_t)st0 * 4 + grp) * m_pad + col) * 16;
      dst[u] = panel * kPanelBytes + grp * 2048 + half * 1024;
    }
  }

  // Stage st0 + ks of the item into an LDS buffer (64 m_pad bytes per stage).
  __device__ __forceinline__ void issue(char* buf, int64_t m_pad, int ks) const {
    const int64_t off = (int64_t)ks * 64 * m_pad;
#pragma unroll
    for (int u = 0; u < 32 / NW; ++u)
      __builtin_amdgcn_global_load_lds(src[u] + off, (lds_ptr_t)(buf + dst[u]), 16, 0, 0);
  }
};

// Rank-one term added to every entry of a low-precision sample-space Gram.
// T_b = dO_b dO_b^H / n_s has the constant vector 1 as an exact null vector
// (the columns of dO are centred).  FP32 accumulation over the n_b terms of each
// entry leaves an error of order sqrt(n_b) 2^-24 times the diagonal, which can
// exceed lambda along 1 and spoil the factorisation there.  Adding
// (t_b / n_s) 11^T / n_s (t_b = tr T_b, so the added eigenvalue is the mean
// diagonal) moves that direction well away from the rounding level.  The right
// side dE and the solution z are orthogonal to 1, and the shifted operator maps
// 1 to lambda 1, so the preconditioner changes only along a direction the
// iteration never needs.
__device__ __forceinline__ double sample_form_deflation(const BlockDev& B, const char* ws) {
  if (B.form != FORM_S || B.prec == PREC_FP64) return 0.0;
  const double m = (double)B.m;
  return *ws_at<double>(ws, B.tr_off) / (m * m);
}

template <int PREC>
__global__ void __launch_bounds__(64 * GramShape<PREC>::NW) k_gram(const GramItem* items, const int32_t* xcd_start, const int32_t* xcd_len,
                                              const BlockDev* blocks, char* ws, double2* part) {
  __shared__ __attribute__((aligned(16))) char lds[3][kStageBytes];
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  if (jx >= xcd_len[x]) return;
  const GramItem it = items[xcd_start[x] + jx];
  const BlockDev B = blocks[it.g];
  const char* re_base = ws + B.pack_off;
  const char* im_base = re_base + B.K_pad * B.m_pad * prec_bytes(PREC);

  constexpr int NW = GramShape<PREC>::NW, SB = GramShape<PREC>::SB, LPW = GramShape<PREC>::LPW;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w / (NW / 2), wc = w % (NW / 2);
  const int l16 = lane & 15, lg = lane >> 4;

  typedef typename std::conditional<PREC == PREC_FP64, d4v, f4v>::type acc_t;
  acc_t accR[4][SB], accI[4][SB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }

  const int ns = it.s1 - it.s0;
  GramLoads<NW> ld;
  ld.init(re_base, im_base, B.m_pad, it.ti, it.tj, it.s0);
  ld.issue(lds[0], B.m_pad, 0);
  if (ns > 1) ld.issue(lds[1], B.m_pad, 1);
  for (int k = 0; k < ns; ++k) {
    // this wave's loads of stage k have landed (stage k+1 may still be in flight)
    if (k + 1 < ns) QGT_WAIT_VMCNT(LPW);
    else QGT_WAIT_VMCNT(0);
    // every wave's loads of stage k have landed, and every wave has finished
    // reading stage k-1, whose buffer is refilled next
    __builtin_amdgcn_s_barrier();
    if (k + 2 < ns) ld.issue(lds[(k + 2) % 3], B.m_pad, k + 2);
    __builtin_amdgcn_iglp_opt(0);  // let the scheduler interleave the stage's LDS reads with its MFMAs
    const char* P = lds[k % 3];
    const int offA = lg * 2048 + (64 * wr + l16) * 16;
    const int offB = lg * 2048 + (16 * SB * wc + l16) * 16;
    if constexpr (PREC == PREC_BF16) {
      bf8v aR[4], aI[4], bR[SB], bI[SB];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        aR[s] = *reinterpret_cast<const bf8v*>(P + 0 * kPanelBytes + offA + s * 256);
        aI[s] = bf8_neg(*reinterpret_cast<const bf8v*>(P + 1 * kPanelBytes + offA + s * 256));  // -I_i
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        bR[s] = *reinterpret_cast<const bf8v*>(P + 2 * kPanelBytes + offB + s * 256);
        bI[s] = *reinterpret_cast<const bf8v*>(P + 3 * kPanelBytes + offB + s * 256);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR[a], bR[b], accR[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aR[a], bI[b], accI[a][b], 0, 0, 0);
          accI[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aI[a], bR[b], accI[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int b = 0; b < SB; ++b) bI[b] = bf8_neg(bI[b]);  // -I_j, so that (-I_i)(-I_j) adds I_i^T I_j to Re
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < SB; ++b)
          accR[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aI[a], bI[b], accR[a][b], 0, 0, 0);
    } else {
      constexpr int G = pack_group(PREC);
      typedef typename std::conditional<PREC == PREC_FP64, double, float>::type T;
      typedef T vG __attribute__((ext_vector_type(G)));
      vG aR[4], aI[4], bR[SB], bI[SB];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        aR[s] = *reinterpret_cast<const vG*>(P + 0 * kPanelBytes + offA + s * 256);
        aI[s] = *reinterpret_cast<const vG*>(P + 1 * kPanelBytes + offA + s * 256);
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        bR[s] = *reinterpret_cast<const vG*>(P + 2 * kPanelBytes + offB + s * 256);
        bI[s] = *reinterpret_cast<const vG*>(P + 3 * kPanelBytes + offB + s * 256);
      }
#pragma unroll
      for (int e = 0; e < G; ++e)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < SB; ++b) {
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

  // Epilogue.  Output layout of the 16x16 MFMA tiles: lane l, register r holds
  // row 4*(l/16)+r (FP32/BF16) or 4*r+l/16 (FP64), column l%16.  Stored as
  // complex FP32 where the block is factored in FP32, else complex FP64.
  double2* A = ws_at<double2>(ws, B.mat_off);
  fv2* Af = ws_at<fv2>(ws, B.mat_off);
  const double defl = it.slot >= 0 ? 0.0 : sample_form_deflation(B, ws);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < SB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int iloc = 64 * wr + 16 * a + (PREC == PREC_FP64 ? 4 * r + lg : 4 * lg + r);
        const int jloc = 16 * SB * wc + 16 * b + l16;
        double re = (double)accR[a][b][r], im = (double)accI[a][b][r];
        if (it.slot >= 0) {
          part[((int64_t)it.slot * 128 + iloc) * 128 + jloc] = make_double2(re, im);
        } else {
          const int64_t R = (int64_t)it.ti * 128 + iloc, Cc = (int64_t)it.tj * 128 + jloc;
          re *= B.inv_ns;
          im *= B.inv_ns;
          if (R < B.m && Cc < B.m) re += defl;
          if (R == Cc) {
            re = R < B.m ? re + B.lambda : 1.0;
            im = 0.0;
          }
          if (PREC == PREC_BF16 && B.fact32) Af[R * B.m_pad + Cc] = fv2{(float)re, (float)im};
          else A[R * B.m_pad + Cc] = make_double2(re, im);
        }
      }
}

// ---------------------------------------------------------------------------
// Wide tiles for large BF16 blocks (m_pad a multiple of 256): 256x128 output
// tiles, 8 waves in a 4x2 arrangement of 64x64 sub-tiles, each a 2x2 grid of
// 32x32 MFMA blocks (v_mfma_f32_32x32x16_bf16, which issues a third more
// flops per cycle than the 16x16x32 form).  Against the
// 128x128 kernel this reads a third less LDS and a quarter less global operand
// per flop.  Stage: A panel (256 columns) Re and Im, 16 KB each, then B panel
// (128 columns) Re and Im, 8 KB each, for four k-groups; three stages in LDS.
constexpr int kWideStageBytes = 49152;

// The six 1 KB loads each wave issues per stage (global -> LDS): the lane's
// source address for the item's first stage, and the uniform destination
// offset within a stage buffer.  Computed once per item, so that issuing a
// stage costs an address increment and the load per slot (the wave index is
// made provably uniform: the LDS destination is taken from a scalar
// register, so it must not need a per-lane loop).
struct WideLoads {
  const char* src[6];
  int dst[6];
};

__device__ __forceinline__ void wide_loads_init(WideLoads& L, const char* re_base, const char* im_base,
                                                int64_t m_pad, int ti, int tj, int st0) {
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int qi = w * 6 + u;  // 0..47, wave-uniform
    int64_t col;
    int plane, grp;
    if (qi < 32) {  // A panels: plane, k-group, quarter of 64 columns
      plane = qi >> 4;
      grp = (qi >> 2) & 3;
      const int qq = qi & 3;
      col = (int64_t)ti * 256 + qq * 64 + lane;
      L.dst[u] = plane * 16384 + grp * 4096 + qq * 1024;
    } else {  // B panels: plane, k-group, half of 64 columns
      const int b = qi - 32;
      plane = b >> 3;
      grp = (b >> 1) & 3;
      const int hh = b & 1;
      col = (int64_t)tj * 128 + hh * 64 + lane;
      L.dst[u] = 32768 + plane * 8192 + grp * 2048 + hh * 1024;
    }
    L.src[u] = (plane ? im_base : re_base) + (((int64_t)st0 * 4 + grp) * m_pad + col) * 16;
  }
}

// Stage st0 + ks of the item into an LDS buffer (a stage is 4 k-groups of
// m_pad 16-byte entries per plane: 64 m_pad bytes further on).
__device__ __forceinline__ void wide_loads_issue(const WideLoads& L, char* buf, int64_t m_pad, int ks) {
  const int64_t off = (int64_t)ks * 64 * m_pad;
#pragma unroll
  for (int u = 0; u < 6; ++u) __builtin_amdgcn_global_load_lds(L.src[u] + off, (lds_ptr_t)(buf + L.dst[u]), 16, 0, 0);
}

// The operand fragments of one 16-deep k-step of a wave's 64x64 sub-tile:
// two 32-row slices of the row panel (Re, -Im) and two 32-column slices of
// the column panel (Re, Im).
struct WideFrag {
  bf8v aR[2], aI[2], bR[2], bI[2];
};

// v_mfma_f32_32x32x16_bf16: lane l holds 8 consecutive k of row (or column)
// l % 32, k-group (l / 32) of the k-step.
// The stage layout: the row panel's Re then Im planes, each of four k-groups
// of AC columns (16 bytes each), then the column panel's Re and Im planes of
// four k-groups of 128 columns.
template <int AC>
__device__ __forceinline__ void wide_frag_read(WideFrag& F, const char* P, int ks, int wr, int wc, int l32, int lh) {
  constexpr int kAGroup = AC * 16, kAPlane = 4 * kAGroup, kB = 2 * kAPlane;
  const int grp = 2 * ks + lh;
  const int offA = grp * kAGroup + (64 * wr + l32) * 16;
  const int offB = kB + grp * 2048 + (64 * wc + l32) * 16;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    F.aR[s] = *reinterpret_cast<const bf8v*>(P + offA + s * 512);
    F.aI[s] = *reinterpret_cast<const bf8v*>(P + kAPlane + offA + s * 512);
    F.bR[s] = *reinterpret_cast<const bf8v*>(P + offB + s * 512);
    F.bI[s] = *reinterpret_cast<const bf8v*>(P + offB + 8192 + s * 512);
  }
}

// The sixteen MFMAs of one k-step: Re += R_i^T R_j + I_i^T I_j, Im += R_i^T I_j
// - I_i^T R_j; the one sign is applied to a fragment in registers (the
// product of the two imaginary fragments needs none).
__device__ __forceinline__ void wide_frag_mfma(const WideFrag& F, f16v (&accR)[2][2], f16v (&accI)[2][2]) {
  bf8v nI[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) nI[s] = bf8_neg(F.aI[s]);  // -I_i
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accR[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.aR[a], F.bR[b], accR[a][b], 0, 0, 0);
      accI[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.aR[a], F.bI[b], accI[a][b], 0, 0, 0);
      accI[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(nI[a], F.bR[b], accI[a][b], 0, 0, 0);
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
      accR[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.aI[a], F.bI[b], accR[a][b], 0, 0, 0);
}

__global__ void __launch_bounds__(512) k_gram_wide(const GramItem* items, const int32_t* xcd_start,
                                                   const int32_t* xcd_len, const BlockDev* blocks, char* ws) {
  __shared__ __attribute__((aligned(16))) char lds[3][kWideStageBytes];
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  if (jx >= xcd_len[x]) return;
  const GramItem it = items[xcd_start[x] + jx];
  const BlockDev B = blocks[it.g];
  const char* re_base = ws + B.pack_off;
  const char* im_base = re_base + B.K_pad * B.m_pad * 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;

  // v_mfma_f32_32x32x16_bf16: lane l holds 8 consecutive k of row (or column)
  // l % 32, k-group (l / 32) of the k-step; output register r of lane l is
  // entry (8 (r / 4) + 4 (l / 32) + r % 4, l % 32) of the 32x32 block.
  f16v accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }
  const int l32 = lane & 31, lh = lane >> 5;

  const int ns = it.s1 - it.s0;
  WideLoads ld;
  wide_loads_init(ld, re_base, im_base, B.m_pad, it.ti, it.tj, it.s0);
  wide_loads_issue(ld, lds[0], B.m_pad, 0);
  if (ns > 1) wide_loads_issue(ld, lds[1], B.m_pad, 1);
  // Software pipeline across the stage barrier: the MFMAs of the second
  // k-step of stage k-1 (fragments already in registers) run after barrier k,
  // while the fragments of the first k-step of stage k are read from LDS, so
  // the matrix pipe is not idle for an LDS round trip after every barrier.
  WideFrag X, Y;
  for (int k = 0; k < ns; ++k) {
    // this wave's six loads of stage k have landed (stage k+1 may be in flight)
    if (k + 1 < ns) QGT_WAIT_VMCNT(6);
    else QGT_WAIT_VMCNT(0);
    // every wave's loads of stage k have landed, and every wave's LDS reads of
    // stage k-1 have completed (waited below), so its buffer can be refilled
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_iglp_opt(0);  // let the scheduler interleave LDS reads with the MFMAs
    const char* P = lds[k % 3];
    wide_frag_read<256>(X, P, 0, wr, wc, l32, lh);
    if (k > 0) wide_frag_mfma(Y, accR, accI);
    wide_frag_read<256>(Y, P, 1, wr, wc, l32, lh);
    // stage k+2's loads go out after this stage's fragment reads: issued
    // straight after the barrier they held back the reads the first MFMAs
    // wait for (the buffer they fill was last read before the barrier)
    if (k + 2 < ns) wide_loads_issue(ld, lds[(k + 2) % 3], B.m_pad, k + 2);
    wide_frag_mfma(X, accR, accI);
    QGT_WAIT_LGKMCNT0();  // the reads of stage k are complete before the next barrier
  }
  if (ns > 0) wide_frag_mfma(Y, accR, accI);

  fv2* Af = ws_at<fv2>(ws, B.mat_off);      // complex FP32 storage (FP32 factor)
  double2* A = ws_at<double2>(ws, B.mat_off);  // complex FP64 storage (FP64 factor)
  const double defl = sample_form_deflation(B, ws);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t R = (int64_t)it.ti * 256 + 64 * wr + 32 * a + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int64_t Cc = (int64_t)it.tj * 128 + 64 * wc + 32 * b + l32;
        double re = (double)accR[a][b][r] * B.inv_ns, im = (double)accI[a][b][r] * B.inv_ns;
        if (R < B.m && Cc < B.m) re += defl;
        if (R == Cc) {
          re = R < B.m ? re + B.lambda : 1.0;
          im = 0.0;
        }
        if (B.fact32) Af[R * B.m_pad + Cc] = fv2{(float)re, (float)im};
        else A[R * B.m_pad + Cc] = make_double2(re, im);
      }
}

// ---------------------------------------------------------------------------
// 128x128 BF16 tiles with two workgroups per CU: 4 waves in a 2x2
// arrangement of 64x64 sub-tiles (the same 2x2 grids of 32x32x16 MFMAs as the
// wide kernel) and a two-stage 32 KB LDS ring, so that two workgroups fit on a
// CU (64 KB of LDS and two waves per SIMD each).  The two workgroups on a CU
// have independent barriers: while one waits at its stage barrier the other
// keeps the matrix cores busy.  Stage: row panel (128 columns) Re and Im,
// 8 KB each, then column panel Re and Im, 8 KB each, for four k-groups.
constexpr int kDuoStageBytes = 32768;

// The eight 1 KB loads each wave issues per stage, described once per tile
// as for the wide kernel.
struct DuoLoads {
  const char* src[8];
  int dst[8];
};

__device__ __forceinline__ void duo_loads_init(DuoLoads& L, const char* re_base, const char* im_base, int64_t m_pad,
                                               int ti, int tj, int st0) {
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int qi = w * 8 + u;      // 0..31, wave-uniform
    const int panel = qi >> 3;     // Re_i, Im_i, Re_j, Im_j
    const int grp = (qi >> 1) & 3; // k-group
    const int half = qi & 1;       // columns 0-63 or 64-127 of the tile
    const int tile = panel < 2 ? ti : tj;
    const int64_t col = (int64_t)tile * 128 + half * 64 + lane;
    L.src[u] = ((panel & 1) ? im_base : re_base) + (((int64_t)st0 * 4 + grp) * m_pad + col) * 16;
    L.dst[u] = panel * 8192 + grp * 2048 + half * 1024;
  }
}

__device__ __forceinline__ void duo_loads_issue(const DuoLoads& L, char* buf, int64_t m_pad, int ks) {
  const int64_t off = (int64_t)ks * 64 * m_pad;
#pragma unroll
  for (int u = 0; u < 8; ++u) __builtin_amdgcn_global_load_lds(L.src[u] + off, (lds_ptr_t)(buf + L.dst[u]), 16, 0, 0);
}

__global__ void __launch_bounds__(256, 2) k_gram_duo(const GramItem* items, const int32_t* xcd_start,
                                                     const int32_t* xcd_len, const BlockDev* blocks, char* ws) {
  __shared__ __attribute__((aligned(16))) char lds[2][kDuoStageBytes];
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  if (jx >= xcd_len[x]) return;
  const GramItem it = items[xcd_start[x] + jx];
  const BlockDev B = blocks[it.g];
  const char* re_base = ws + B.pack_off;
  const char* im_base = re_base + B.K_pad * B.m_pad * 2;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int l32 = lane & 31, lh = lane >> 5;

  f16v accR[2][2], accI[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) { accR[a][b][r] = 0; accI[a][b][r] = 0; }

  const int ns = it.s1 - it.s0;
  DuoLoads ld;
  duo_loads_init(ld, re_base, im_base, B.m_pad, it.ti, it.tj, it.s0);
  if (ns > 0) duo_loads_issue(ld, lds[0], B.m_pad, 0);
  // as in the wide kernel, the MFMAs of the second k-step of stage k-1 run
  // after barrier k, over the LDS reads of stage k
  WideFrag X, Y;
  for (int k = 0; k < ns; ++k) {
    // this wave's loads of stage k have landed (the only stage in flight)
    QGT_WAIT_VMCNT(0);
    // every wave's loads of stage k have landed, and every wave's LDS reads of
    // stage k-1 have completed (waited below), so its buffer can be refilled
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_iglp_opt(0);
    const char* P = lds[k & 1];
    wide_frag_read<128>(X, P, 0, wr, wc, l32, lh);
    if (k > 0) wide_frag_mfma(Y, accR, accI);
    wide_frag_read<128>(Y, P, 1, wr, wc, l32, lh);
    if (k + 1 < ns) duo_loads_issue(ld, lds[(k + 1) & 1], B.m_pad, k + 1);  // as in the wide kernel
    wide_frag_mfma(X, accR, accI);
    QGT_WAIT_LGKMCNT0();
  }
  if (ns > 0) wide_frag_mfma(Y, accR, accI);

  fv2* Af = ws_at<fv2>(ws, B.mat_off);
  double2* A = ws_at<double2>(ws, B.mat_off);
  const double defl = sample_form_deflation(B, ws);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t R = (int64_t)it.ti * 128 + 64 * wr + 32 * a + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int64_t Cc = (int64_t)it.tj * 128 + 64 * wc + 32 * b + l32;
        double re = (double)accR[a][b][r] * B.inv_ns, im = (double)accI[a][b][r] * B.inv_ns;
        if (R < B.m && Cc < B.m) re += defl;
        if (R == Cc) {
          re = R < B.m ? re + B.lambda : 1.0;
          im = 0.0;
        }
        if (B.fact32) Af[R * B.m_pad + Cc] = fv2{(float)re, (float)im};
        else A[R * B.m_pad + Cc] = make_double2(re, im);
      }
}

// Ordered sum of split-K partial tiles, then the same epilogue.
// 64 workgroups per tile, one entry per thread.
__global__ void __launch_bounds__(256) k_gram_splitk_reduce(const SplitItem* items, const BlockDev* blocks, char* ws,
                                                            const double2* part) {
  const SplitItem it = items[blockIdx.x >> 6];
  const BlockDev B = blocks[it.g];
  {
    const int idx = (blockIdx.x & 63) * 256 + threadIdx.x;
    const int iloc = idx >> 7, jloc = idx & 127;
    double2 s = part[(int64_t)it.slot0 * 16384 + idx];
    for (int q = 1; q < it.nsplit; ++q) s = cadd(s, part[(int64_t)(it.slot0 + q) * 16384 + idx]);
    const int64_t R = (int64_t)it.ti * 128 + iloc, Cc = (int64_t)it.tj * 128 + jloc;
    double re = s.x * B.inv_ns, im = s.y * B.inv_ns;
    if (R < B.m && Cc < B.m) re += sample_form_deflation(B, ws);
    if (R == Cc) {
      re = R < B.m ? re + B.lambda : 1.0;
      im = 0.0;
    }
    if (B.fact32) ws_at<fv2>(ws, B.mat_off)[R * B.m_pad + Cc] = fv2{(float)re, (float)im};
    else ws_at<double2>(ws, B.mat_off)[R * B.m_pad + Cc] = make_double2(re, im);
  }
}

void launch_gram_wide(const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                      const BlockDev* blocks, char* ws, hipStream_t s) {
  if (maxlen <= 0) return;
  hipLaunchKernelGGL(k_gram_wide, dim3(8 * maxlen), dim3(512), 0, s, items, xcd_start, xcd_len, blocks, ws);
}

void launch_gram_duo(const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                     const BlockDev* blocks, char* ws, hipStream_t s) {
  if (maxlen <= 0) return;
  hipLaunchKernelGGL(k_gram_duo, dim3(8 * maxlen), dim3(256), 0, s, items, xcd_start, xcd_len, blocks, ws);
}

void launch_gram(int prec, const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                 const BlockDev* blocks, char* ws, double2* part, hipStream_t s) {
  if (maxlen <= 0) return;
  dim3 grid(8 * maxlen);
  if (prec == PREC_FP64)
    hipLaunchKernelGGL(k_gram<PREC_FP64>, grid, dim3(512), 0, s, items, xcd_start, xcd_len, blocks, ws, part);
  else if (prec == PREC_FP32)
    hipLaunchKernelGGL(k_gram<PREC_FP32>, grid, dim3(256), 0, s, items, xcd_start, xcd_len, blocks, ws, part);
  else
    hipLaunchKernelGGL(k_gram<PREC_BF16>, grid, dim3(512), 0, s, items, xcd_start, xcd_len, blocks, ws, part);
}

void launch_gram_splitk_reduce(const SplitItem* items, int n, const BlockDev* blocks, char* ws, const double2* part,
                               hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gram_splitk_reduce, dim3(n * 64), dim3(256), 0, s, items, blocks, ws, part);
}

}  // namespace qgt
