// Device formation of O, the per-sample log-derivatives O_k(x) = d log psi(x) /
// d theta_k (paper, Sec. 2, the definition that follows Eq. 2), for the
// networks that stand in for the paper's Vision Transformer: an RBM and a
// feed-forward network of dense logcosh layers (optionally with a dense
// readout).  All networks are holomorphic in their complex parameters, so the
// chain rule uses plain transposes.
//
// Two kinds of kernels:
//   * k_dense<MODE>: the batched dense-layer products of the forward pass
//     (z = W h + b over all samples, with tanh(z) and logcosh(z) in the
//     epilogue) and of the backward pass (the derivative reaching h^{l-1} is
//     W^T g^l, times tanh(z^{l-1})).  FP64 on the vector ALUs: 64x32 output
//     tiles, 16-deep k-stages in LDS.  The products are small next to the
//     write of O (they read n_s x width activations, O holds n_s x n_p).
//   * k_jac_rows<DT>: writes the rows of O from the per-sample vectors, every
//     entry a product g_j * h_i of two FP64 complex numbers rounded once to
//     the output type.  HBM-bound: one coalesced pass of stores over O.
#include <hip/hip_runtime.h>

#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

namespace {

constexpr double kLog2 = 0.69314718055994530942;

// tanh of a complex number: with z = a + ib,
//   tanh z = (sinh a cosh a + i sin b cos b) / (sinh^2 a + cos^2 b),
// a denominator of two non-negative terms (no cancellation away from the
// poles a = 0, b = pi/2 + k pi).  For |a| > 20 the real part is sign(a) to
// FP64 precision and the imaginary part 2 sin(2b) exp(-2|a|).
__device__ dv2 ctanh(dv2 z) {
  const double a = z.x, b = z.y;
  double sb, cb;
  sincos(b, &sb, &cb);
  if (fabs(a) > 20.0) return dv2{copysign(1.0, a), 4.0 * sb * cb * exp(-2.0 * fabs(a))};
  const double sh = sinh(a), ch = cosh(a);
  const double den = fma(sh, sh, cb * cb);
  return dv2{sh * ch / den, sb * cb / den};
}

// log cosh on the fixed branch s z + log1p(exp(-2 s z)) - log 2, s = sign(Re z)
// (s = +1 at Re z = 0).  With w = exp(-2 s z), |w| <= 1:
//   log1p(w) = (1/2) log1p(2 Re w + |w|^2) + i arg(1 + w).
__device__ dv2 clogcosh(dv2 z) {
  const double s = z.x >= 0.0 ? 1.0 : -1.0;
  const double m = exp(-2.0 * fabs(z.x));
  double sn, cs;
  sincos(2.0 * s * z.y, &sn, &cs);
  const double wr = m * cs, wi = -m * sn;
  const double re = 0.5 * log1p(fma(wr, 2.0 + wr, wi * wi));
  const double im = atan2(wi, 1.0 + wr);
  return dv2{fabs(z.x) + re - kLog2, s * z.y + im};
}

__device__ __forceinline__ dv2 vmul(dv2 a, dv2 b) {
  return dv2{fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

constexpr int kDS = 64;   // samples per tile
constexpr int kDO = 32;   // outputs per tile
constexpr int kDK = 16;   // k-stage depth

// MODE 0: forward layer; MODE 1: backward product.  256 threads: thread
// (ty, tx) = (t / 16, t % 16) owns samples ty + 16 i (i < 4) and outputs
// tx + 16 j (j < 2) of the tile.
template <int MODE>
__global__ __launch_bounds__(256) void k_dense(const DenseArgs A) {
  __shared__ dv2 As[kDK][kDS + 1];
  __shared__ dv2 Bs[kDK][kDO + 1];
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * kDS;
  const int o0 = blockIdx.y * kDO;
  dv2 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dv2{0.0, 0.0};

  for (int k0 = 0; k0 < A.n_k; k0 += kDK) {
    // A stage: 16 k x 64 samples, consecutive lanes on consecutive k
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = t + 256 * r, kk = e & 15, ss = e >> 4;
      const int64_t s = s0 + ss;
      const int k = k0 + kk;
      dv2 v = dv2{0.0, 0.0};
      if (s < A.n_s && k < A.n_k) {
        if (A.x) v.x = (double)A.x[s * A.lda + k];
        else v = ((const QGT_GLOBAL dv2*)A.a)[s * A.lda + k];
      }
      As[kk][ss] = v;
    }
    // B stage: 16 k x 32 outputs, consecutive lanes along the contiguous index
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = t + 256 * r;
      int kk, oo;
      if (MODE == 0) { kk = e & 15; oo = e >> 4; }   // W[o][k]: k contiguous
      else { oo = e & 31; kk = e >> 5; }             // W[k][o]: o contiguous
      const int k = k0 + kk, o = o0 + oo;
      dv2 v = dv2{0.0, 0.0};
      if (k < A.n_k && o < A.n_o) v = ((const QGT_GLOBAL dv2*)A.W)[(int64_t)k * A.wk + (int64_t)o * A.wo];
      Bs[kk][oo] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kDK; ++kk) {
      dv2 a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = vfma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t s = s0 + ty + 16 * i;
    if (s >= A.n_s) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int o = o0 + tx + 16 * j;
      if (o >= A.n_o) continue;
      QGT_GLOBAL dv2* tg = (QGT_GLOBAL dv2*)A.tg + s * A.ldt + o;
      if (MODE == 0) {
        const dv2 z = acc[i][j] + ((const QGT_GLOBAL dv2*)A.bias)[o];
        dv2 th = ctanh(z);
        if (A.scale) th = vmul(th, ((const QGT_GLOBAL dv2*)A.scale)[o]);
        *tg = th;
        if (A.h) ((QGT_GLOBAL dv2*)A.h)[s * A.ldt + o] = clogcosh(z);
      } else {
        *tg = vmul(*tg, acc[i][j]);
      }
    }
  }
}

template <int DT>
__device__ __forceinline__ void store_o(QGT_GLOBAL char* orow, int64_t c, dv2 v) {
  if constexpr (DT == 0) ((QGT_GLOBAL fv2*)orow)[c] = fv2{(float)v.x, (float)v.y};
  else ((QGT_GLOBAL dv2*)orow)[c] = v;
}

// One workgroup writes kJacChunk consecutive columns of one row of O; lane t
// takes columns t, t + 256, ... (coalesced stores).  The segment of a column
// is found by a scan of the (at most kJacMaxSegs) segment starts; within an
// OUTER segment the column e splits as e = j n_in + i by a multiply-shift
// (exact for e < 2^24 and n_in < 2^16, which the host checks).
template <int DT>
__global__ __launch_bounds__(256) void k_jac_rows(const JacArgs A) {
  const int64_t row = blockIdx.x / A.chunks;
  const int64_t c0 = (int64_t)(blockIdx.x % A.chunks) * kJacChunk;
  if (row >= A.n_s) return;
  QGT_GLOBAL char* orow = (QGT_GLOBAL char*)A.O + row * A.ldo * (DT == 0 ? 8 : 16);
  auto vin = [&](int layer, uint32_t i) -> dv2 {
    if (layer == 0) return dv2{(double)A.x[row * A.ldx + i], 0.0};
    return ((const QGT_GLOBAL dv2*)A.v[layer])[row * A.ld[layer] + i];
  };
  for (int r = 0; r < kJacChunk / 256; ++r) {
    const int64_t c = c0 + threadIdx.x + 256 * r;
    if (c >= A.n_p) break;
    int si = 0;
    while (si + 1 < A.nseg && c >= A.seg[si + 1].off) ++si;
    const JacSeg& S = A.seg[si];
    const uint32_t e = (uint32_t)(c - S.off);
    dv2 val;
    if (S.kind == JAC_OUTER) {
      const QGT_GLOBAL dv2* grow = (const QGT_GLOBAL dv2*)A.g[S.g_layer] + row * A.ld[S.g_layer];
      const uint32_t nprod = (uint32_t)S.n_out * (uint32_t)S.n_in;
      if (e < nprod) {
        const uint32_t j = (uint32_t)(((uint64_t)e * S.magic) >> 40);
        val = vmul(grow[j], vin(S.v_layer, e - j * (uint32_t)S.n_in));
      } else {
        val = grow[e - nprod];
      }
    } else {
      val = e < (uint32_t)S.n_in ? vin(S.v_layer, e) : dv2{1.0, 0.0};
    }
    store_o<DT>(orow, c, val);
  }
}

}  // namespace

void launch_dense(int mode, const DenseArgs& a, hipStream_t s) {
  // samples on x (up to 2^18 tiles), outputs on y (at most 2048 tiles)
  const dim3 grid((unsigned)((a.n_s + kDS - 1) / kDS), (unsigned)((a.n_o + kDO - 1) / kDO));
  if (mode == 0) hipLaunchKernelGGL(k_dense<0>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_dense<1>, grid, dim3(256), 0, s, a);
}

void launch_jac_rows(int dt, const JacArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.n_s * a.chunks));
  if (dt == 0) hipLaunchKernelGGL(k_jac_rows<0>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_jac_rows<1>, grid, dim3(256), 0, s, a);
}

}  // namespace qgt
