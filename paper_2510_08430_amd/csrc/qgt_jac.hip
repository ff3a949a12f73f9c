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
//     W^T g^l, times tanh(z^{l-1})).  FP64 matrix cores (four real
//     16x16x4 MFMAs per complex product), 64x32 (or 32x32) output tiles,
//     16-deep k-stages in LDS.  The products are small next to the
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

constexpr int kDO = 32;   // outputs per tile
constexpr int kDK = 16;   // k-stage depth

// MODE 0: forward layer; MODE 1: backward product.  DS samples per tile (64,
// or 32 when the layer would otherwise give fewer than two workgroups per
// CU) by 32 outputs; four waves, each owning 16 samples by 16 NT outputs
// (NT = DS / 32).  The complex products run as four real FP64 MFMAs
// (v_mfma_f64_16x16x4_f64): Re += a.re b.re - a.im b.im, Im += a.im b.re +
// a.re b.im.  Operand layout of the 16x16x4 instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; result element r of lane l is
// D[4 r + l / 16][l % 16].
__device__ __forceinline__ d4v mfma64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int MODE, int DS>
__global__ __launch_bounds__(256) void k_dense(const DenseArgs A) {
  constexpr int NI = DS / 16;        // A-stage loads per thread
  constexpr int NT = DS / 32;        // 16-output tiles per wave
  __shared__ dv2 As[kDK][DS + 1];
  __shared__ dv2 Bs[kDK][kDO + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rb = w % (DS / 16);      // the wave's 16-sample block
  const int cb = (w / (DS / 16)) * NT;  // its first 16-output tile
  const int64_t s0 = (int64_t)blockIdx.x * DS;
  const int o0 = blockIdx.y * kDO;
  d4v cr[NT], ci[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) cr[j] = ci[j] = d4v{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < A.n_k; k0 += kDK) {
    // A stage: 16 k x DS samples, consecutive lanes on consecutive k
#pragma unroll
    for (int r = 0; r < NI; ++r) {
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
    for (int ks = 0; ks < kDK / 4; ++ks) {
      const int kk = 4 * ks + lk;
      const dv2 a = As[kk][16 * rb + li];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const dv2 b = Bs[kk][16 * (cb + j) + li];
        cr[j] = mfma64(a.x, b.x, cr[j]);
        cr[j] = mfma64(-a.y, b.y, cr[j]);
        ci[j] = mfma64(a.y, b.x, ci[j]);
        ci[j] = mfma64(a.x, b.y, ci[j]);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t s = s0 + 16 * rb + 4 * r + lk;
    if (s >= A.n_s) continue;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int o = o0 + 16 * (cb + j) + li;
      if (o >= A.n_o) continue;
      const dv2 acc = dv2{cr[j][r], ci[j][r]};
      QGT_GLOBAL dv2* tg = (QGT_GLOBAL dv2*)A.tg + s * A.ldt + o;
      if (MODE == 0) {
        const dv2 z = acc + ((const QGT_GLOBAL dv2*)A.bias)[o];
        dv2 th = ctanh(z);
        if (A.scale) th = vmul(th, ((const QGT_GLOBAL dv2*)A.scale)[o]);
        *tg = th;
        if (A.h) ((QGT_GLOBAL dv2*)A.h)[s * A.ldt + o] = clogcosh(z);
      } else {
        *tg = vmul(*tg, acc);
      }
    }
  }
}

template <int DT>
__device__ __forceinline__ void store_o(QGT_GLOBAL char* orow, int64_t c, dv2 v) {
  if constexpr (DT == 0) ((QGT_GLOBAL fv2*)orow)[c] = fv2{(float)v.x, (float)v.y};
  else ((QGT_GLOBAL dv2*)orow)[c] = v;
}

// One workgroup writes one task of one row of O.  In an OUTER task the
// columns of product rows [ja, jb) are contiguous: with n_in < 256, lane t
// takes row ja + t / n_in + k rpi and column t % n_in (rpi = 256 / n_in rows
// per pass), with n_in >= 256 it takes columns t, t + 256, ... of every row;
// either way consecutive lanes store consecutive columns, the lane's v entry
// stays in a register and the division by n_in happens once per lane.  The
// segment of the task is found by a loop over the segment table that depends
// on the workgroup only (scalar loads).
template <int DT>
__global__ __launch_bounds__(256) void k_jac_rows(const JacArgs A) {
  const int64_t row = blockIdx.x / A.tasks;
  const int32_t task = (int32_t)(blockIdx.x - row * A.tasks);
  if (row >= A.n_s) return;
  QGT_GLOBAL char* orow = (QGT_GLOBAL char*)A.O + row * A.ldo * (DT == 0 ? 8 : 16);
  int si = 0;
  while (si + 1 < A.nseg && task >= A.seg[si + 1].task0) ++si;
  const JacSeg S = A.seg[si];
  const int t = threadIdx.x;
  const QGT_GLOBAL dv2* vrow = S.v_layer > 0 ? (const QGT_GLOBAL dv2*)A.v[S.v_layer] + row * A.ld[S.v_layer] : nullptr;
  const QGT_GLOBAL int8_t* xrow = (const QGT_GLOBAL int8_t*)A.x + row * A.ldx;
  auto vin = [&](int i) -> dv2 {
    if (S.v_layer == 0) return dv2{(double)xrow[i], 0.0};
    return vrow[i];
  };
  if (S.kind == JAC_COPY) {
    for (int e = t; e < S.n_in + S.tail_one; e += 256) store_o<DT>(orow, S.off + e, e < S.n_in ? vin(e) : dv2{1.0, 0.0});
    return;
  }
  const QGT_GLOBAL dv2* grow = (const QGT_GLOBAL dv2*)A.g[S.g_layer] + row * A.ld[S.g_layer];
  const int32_t blk = task - S.task0;
  const int32_t ja = blk * S.jrows;
  const int32_t jb = ja + S.jrows < S.n_out ? ja + S.jrows : S.n_out;
  // the task's derivatives g[ja..jb) in LDS (one coalesced load), so that the
  // store loop below waits on no global load
  __shared__ dv2 gsh[kJacMaxTaskRows];
  for (int e = t; e < jb - ja; e += 256) gsh[e] = grow[ja + e];
  __syncthreads();
  if (S.n_in < 256) {
    const int jj = t / S.n_in, i = t - jj * S.n_in;
    if (jj < S.rpi) {
      const dv2 v = vin(i);
      for (int j = ja + jj; j < jb; j += S.rpi)
        store_o<DT>(orow, S.off + (int64_t)j * S.n_in + i, vmul(gsh[j - ja], v));
    }
  } else {
    const dv2 v0 = vin(t);
    const dv2 v1 = t + 256 < S.n_in ? vin(t + 256) : dv2{0.0, 0.0};
    for (int j = ja; j < jb; ++j) {
      const dv2 g = gsh[j - ja];
      const int64_t base = S.off + (int64_t)j * S.n_in;
      store_o<DT>(orow, base + t, vmul(g, v0));
      if (t + 256 < S.n_in) store_o<DT>(orow, base + t + 256, vmul(g, v1));
      for (int i = t + 512; i < S.n_in; i += 256) store_o<DT>(orow, base + i, vmul(g, vin(i)));
    }
  }
  if (jb == S.n_out) {  // the last task of the segment also writes the bias part
    const int64_t base = S.off + (int64_t)S.n_out * S.n_in;
    for (int j = t; j < S.n_out; j += 256) store_o<DT>(orow, base + j, grow[j]);
  }
}


// ---------------------------------------------------------------------------
// Periodic 3x3 convolutions (CNN).  Site s = y * side + x; offset k % 9 =
// 3 dy + dx.  The forward gather reads the input at (y + dy - 1, x + dx - 1),
// the backward gather the derivative at (y - dy + 1, x - dx + 1), both modulo
// side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int conv_nbr(int site, int d, int side, int sign) {
  const int y = site / side, x = site - y * side;
  const int dy = d / 3, dx = d - 3 * dy;
  int yy = y + sign * (dy - 1), xx = x + sign * (dx - 1);
  yy = yy < 0 ? yy + side : (yy >= side ? yy - side : yy);
  xx = xx < 0 ? xx + side : (xx >= side ? xx - side : xx);
  return yy * side + xx;
}

constexpr int kCO = 16;   // output channels per tile

// 64 rows (sample, site) by 16 output channels per workgroup; four waves of
// 16 rows; FP64 MFMA as in k_dense, the A operand gathered from the sample's
// channel-major activation array through the periodic neighbour map.
template <int MODE>
__global__ __launch_bounds__(256) void k_conv(const ConvArgs A) {
  __shared__ dv2 As[kDK][64 + 1];
  __shared__ dv2 Bs[kDK][kCO + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int S = A.side * A.side;
  const int64_t nrows = A.n_s * S;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int o0 = blockIdx.y * kCO;
  const int cin_a = MODE == 0 ? A.cin : A.cout;   // channels of the gathered array
  d4v cr = d4v{0.0, 0.0, 0.0, 0.0}, ci = d4v{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < A.n_k; k0 += kDK) {
    // consecutive lanes on consecutive rows (sites) for one k: the gathered
    // addresses are contiguous apart from the lattice wrap
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = t + 256 * r, kk = e >> 6, rr = e & 63;
      const int64_t row = r0 + rr;
      const int k = k0 + kk;
      dv2 v = dv2{0.0, 0.0};
      if (row < nrows && k < A.n_k) {
        const int64_t smp = row / S;
        const int site = (int)(row - smp * S);
        const int c = k / 9, d = k - 9 * c;
        const int nb = conv_nbr(site, d, A.side, MODE == 0 ? 1 : -1);
        if (MODE == 0 && A.x) v.x = (double)A.x[smp * A.ldx + nb];
        else v = ((const QGT_GLOBAL dv2*)A.a)[(smp * cin_a + c) * S + nb];
      }
      As[kk][rr] = v;
    }
    {
      const int kk = t & 15, oo = t >> 4;   // 16 k x 16 outputs
      const int k = k0 + kk, o = o0 + oo;
      dv2 v = dv2{0.0, 0.0};
      if (k < A.n_k && o < A.n_o) {
        int64_t idx;
        if (MODE == 0) idx = (int64_t)o * A.n_k + k;                       // K[o][c][d], k = 9 c + d
        else idx = ((int64_t)(k / 9) * A.cin + o) * 9 + (k - 9 * (k / 9));  // K[c][o][d]
        v = ((const QGT_GLOBAL dv2*)A.K)[idx];
      }
      Bs[kk][oo] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kDK / 4; ++ks) {
      const int kk = 4 * ks + lk;
      const dv2 a = As[kk][16 * w + li];
      const dv2 b = Bs[kk][li];
      cr = mfma64(a.x, b.x, cr);
      cr = mfma64(-a.y, b.y, cr);
      ci = mfma64(a.y, b.x, ci);
      ci = mfma64(a.x, b.y, ci);
    }
    __syncthreads();
  }

  const int o = o0 + li;
  if (o >= A.n_o) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = r0 + 16 * w + 4 * r + lk;
    if (row >= nrows) continue;
    const int64_t smp = row / S;
    const int site = (int)(row - smp * S);
    const int64_t idx = (smp * A.n_o + o) * S + site;
    const dv2 acc = dv2{cr[r], ci[r]};
    QGT_GLOBAL dv2* tg = (QGT_GLOBAL dv2*)A.tg + idx;
    if (MODE == 0) {
      const dv2 z = acc + ((const QGT_GLOBAL dv2*)A.bias)[o];
      *tg = ctanh(z);
      if (A.h) ((QGT_GLOBAL dv2*)A.h)[idx] = clogcosh(z);
    } else {
      *tg = vmul(*tg, acc);
    }
  }
}

// Kernel and bias derivatives of one layer for one sample (blockIdx.x =
// sample, blockIdx.y = layer): dK[c][c'][d] = sum_site g[c][site]
// h[c'][site shifted by d], db[c] = sum_site g[c][site].  The kernel part is
// a product of the sample's g (C x S) with the gathered matrix
// B[site][9 c' + d] = h[c'][site shifted by d] (S x 9 c_in), on the FP64
// matrix cores: wave w takes the 16-column tiles w, w + 4, ...; the
// contraction runs over sites four at a time.  g, h and the neighbour map sit
// in LDS (sized to the layer: dynamic shared memory).  Result rows are output
// channels, columns (c', d): stores along consecutive columns of O.
template <int DT>
__global__ __launch_bounds__(256) void k_conv_dk(const ConvDkArgs A) {
  extern __shared__ __align__(16) char conv_lds[];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t smp = blockIdx.x;
  const ConvDkLayer Ly = A.layer[blockIdx.y];
  const int S = A.side * A.side, C = A.cout, cin = Ly.cin;
  dv2* Gs = (dv2*)conv_lds;                    // C x S
  dv2* Hs = Gs + C * S;                        // cin x S
  int16_t* nbs = (int16_t*)(Hs + cin * S);     // 9 x S
  const QGT_GLOBAL dv2* g = (const QGT_GLOBAL dv2*)Ly.g + smp * C * S;
  for (int e = t; e < C * S; e += 256) Gs[e] = g[e];
  if (Ly.hin) {
    const QGT_GLOBAL dv2* h = (const QGT_GLOBAL dv2*)Ly.hin + smp * cin * S;
    for (int e = t; e < cin * S; e += 256) Hs[e] = h[e];
  } else {
    for (int e = t; e < S; e += 256) Hs[e] = dv2{(double)A.x[smp * A.ldx + e], 0.0};
  }
  for (int e = t; e < 9 * S; e += 256) nbs[e] = (int16_t)conv_nbr(e % S, e / S, A.side, 1);
  __syncthreads();
  QGT_GLOBAL char* orow = (QGT_GLOBAL char*)A.O + smp * A.ldo * (DT == 0 ? 8 : 16);
  const int np = 9 * cin;
  const int ntiles = (np + 15) / 16;
  for (int nt = w; nt < ntiles; nt += 4) {
    const int col = 16 * nt + li;
    const bool cv = col < np;
    const int cp = cv ? col / 9 : 0, d = cv ? col - 9 * cp : 0;
    d4v cr = d4v{0.0, 0.0, 0.0, 0.0}, ci = d4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < S; k0 += 4) {
      const int k = k0 + lk;
      dv2 a = dv2{0.0, 0.0}, b = dv2{0.0, 0.0};
      if (k < S) {
        if (li < C) a = Gs[li * S + k];
        if (cv) b = Hs[cp * S + nbs[d * S + k]];
      }
      cr = mfma64(a.x, b.x, cr);
      cr = mfma64(-a.y, b.y, cr);
      ci = mfma64(a.y, b.x, ci);
      ci = mfma64(a.x, b.y, ci);
    }
    if (cv) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 4 * r + lk;
        if (c < C) store_o<DT>(orow, Ly.off + (int64_t)c * np + col, dv2{cr[r], ci[r]});
      }
    }
  }
  if (t < C) {
    dv2 acc = dv2{0.0, 0.0};
    for (int site = 0; site < S; ++site) acc += Gs[t * S + site];
    store_o<DT>(orow, Ly.off + (int64_t)C * np + t, acc);
  }
}

}  // namespace

void launch_dense(int mode, const DenseArgs& a, hipStream_t s) {
  // samples on x (up to 2^19 tiles), outputs on y (at most 2048 tiles)
  const unsigned oy = (unsigned)((a.n_o + kDO - 1) / kDO);
  const bool small = ((a.n_s + 63) / 64) * oy < 512;
  const dim3 grid((unsigned)((a.n_s + (small ? 31 : 63)) / (small ? 32 : 64)), oy);
  if (small) {
    if (mode == 0) hipLaunchKernelGGL((k_dense<0, 32>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_dense<1, 32>), grid, dim3(256), 0, s, a);
  } else {
    if (mode == 0) hipLaunchKernelGGL((k_dense<0, 64>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_dense<1, 64>), grid, dim3(256), 0, s, a);
  }
}

void launch_conv(int mode, const ConvArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n_s * a.side * a.side + 63) / 64), (unsigned)((a.n_o + kCO - 1) / kCO));
  if (mode == 0) hipLaunchKernelGGL(k_conv<0>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_conv<1>, grid, dim3(256), 0, s, a);
}

void launch_conv_dk(int dt, const ConvDkArgs& a, int n_layers, hipStream_t s) {
  const dim3 grid((unsigned)a.n_s, (unsigned)n_layers);
  const int S = a.side * a.side;
  int cin_max = 1;
  for (int l = 0; l < n_layers; ++l) cin_max = a.layer[l].cin > cin_max ? a.layer[l].cin : cin_max;
  const size_t lds = (size_t)(a.cout + cin_max) * S * 16 + (size_t)9 * S * 2;
  if (dt == 0) hipLaunchKernelGGL(k_conv_dk<0>, grid, dim3(256), lds, s, a);
  else hipLaunchKernelGGL(k_conv_dk<1>, grid, dim3(256), lds, s, a);
}

void launch_jac_rows(int dt, const JacArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.n_s * a.tasks));
  if (dt == 0) hipLaunchKernelGGL(k_jac_rows<0>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_jac_rows<1>, grid, dim3(256), 0, s, a);
}

}  // namespace qgt
