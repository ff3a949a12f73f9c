// Variational Monte Carlo around block SR, for an RBM on the spin-1/2
// Heisenberg chain (paper, Sec. 3, Heisenberg paragraph; Eq. 1 for the local
// energy): a Metropolis sampler of exchange moves, the local energies, and
// the parameter step theta <- theta - eta delta.
//
// RBM: log psi(x) = sum_i a_i x_i + sum_h logcosh(b_h + sum_i W_hi x_i),
// theta = [W (M x N, row-major) | b | a], the same layout as the device
// formation of O.  Configurations are spins +-1; a wave keeps one as a 64-bit
// mask (bit i set for spin +1), so that every lane reads any spin without
// memory traffic, and the lanes run over the hidden units.
#include <hip/hip_runtime.h>

#include "../../include/qgt_vmc.h"
#include "qgt_device.h"
#include "qgt_launch.h"

namespace qgt {

namespace {

constexpr double kLn2 = 0.69314718055994530942;

// logcosh on the branch s z + log1p(exp(-2 s z)) - log 2, s = sign(Re z)
// (the same definition as the formation of O).
__device__ dv2 vlogcosh(dv2 z) {
  const double s = z.x >= 0.0 ? 1.0 : -1.0;
  const double m = exp(-2.0 * fabs(z.x));
  double sn, cs;
  sincos(2.0 * s * z.y, &sn, &cs);
  const double wr = m * cs, wi = -m * sn;
  return dv2{fabs(z.x) + 0.5 * log1p(fma(wr, 2.0 + wr, wi * wi)) - kLn2, s * z.y + atan2(wi, 1.0 + wr)};
}

__device__ __forceinline__ dv2 wave_sum(dv2 v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

struct RbmArgs {
  const double2* theta;
  int32_t N, M;
};

__device__ __forceinline__ double spin(uint64_t mask, int i) { return (mask >> i) & 1 ? 1.0 : -1.0; }

// Hidden field theta_h = b_h + sum_i W_hi x_i of hidden unit h.
__device__ __forceinline__ dv2 hidden_field(const RbmArgs& R, uint64_t mask, int h) {
  const QGT_GLOBAL dv2* th = (const QGT_GLOBAL dv2*)R.theta;
  dv2 acc = th[(int64_t)R.M * R.N + h];
  const QGT_GLOBAL dv2* w = th + (int64_t)h * R.N;
  for (int i = 0; i < R.N; ++i) acc += spin(mask, i) * w[i];
  return acc;
}

// log psi(x with spins i and j exchanged) - log psi(x), for x_i != x_j:
// the changes are dx_i = -2 x_i and dx_j = -2 x_j.  Every lane returns the
// wave's total.
__device__ dv2 exchange_ratio_log(const RbmArgs& R, uint64_t mask, int i, int j, int lane) {
  const QGT_GLOBAL dv2* th = (const QGT_GLOBAL dv2*)R.theta;
  const double dxi = -2.0 * spin(mask, i), dxj = -2.0 * spin(mask, j);
  dv2 part = dv2{0.0, 0.0};
  for (int h = lane; h < R.M; h += 64) {
    const dv2 t = hidden_field(R, mask, h);
    const QGT_GLOBAL dv2* w = th + (int64_t)h * R.N;
    const dv2 t2 = t + dxi * w[i] + dxj * w[j];
    part += vlogcosh(t2) - vlogcosh(t);
  }
  dv2 d = wave_sum(part);
  const QGT_GLOBAL dv2* a = th + (int64_t)R.M * R.N + R.M;
  return d + dxi * a[i] + dxj * a[j];
}

// The same ratio from cached hidden fields t[q] = theta_{lane + 64 q} and
// their logcosh values lc[q] (h < M): the terms and their order are those of
// exchange_ratio_log, so the two give identical results.
constexpr int kHPerLane = 4;   // hidden units cached per lane (M <= 256)
__device__ dv2 exchange_ratio_log_cached(const RbmArgs& R, uint64_t mask, int i, int j, int lane,
                                         const dv2 (&tc)[kHPerLane], const dv2 (&lc)[kHPerLane]) {
  const QGT_GLOBAL dv2* th = (const QGT_GLOBAL dv2*)R.theta;
  const double dxi = -2.0 * spin(mask, i), dxj = -2.0 * spin(mask, j);
  dv2 part = dv2{0.0, 0.0};
#pragma unroll
  for (int q = 0; q < kHPerLane; ++q) {
    const int h = lane + 64 * q;
    if (h < R.M) {
      const QGT_GLOBAL dv2* w = th + (int64_t)h * R.N;
      part += vlogcosh(tc[q] + dxi * w[i] + dxj * w[j]) - lc[q];
    }
  }
  dv2 d = wave_sum(part);
  const QGT_GLOBAL dv2* a = th + (int64_t)R.M * R.N + R.M;
  return d + dxi * a[i] + dxj * a[j];
}

__device__ __forceinline__ uint64_t load_mask(const int8_t* x, int N, int lane) {
  const bool up = lane < N && x[lane] > 0;
  return __ballot(up);
}

// One wave per chain (four chains per workgroup).  Step s proposes the
// exchange of spins pairs[s][c] (a no-op when they are equal or out of
// range) and accepts it when u[s][c] < |psi(x') / psi(x)|^2.
__global__ __launch_bounds__(256) void k_rbm_metropolis(const RbmArgs R, int8_t* x, int64_t ldx, int64_t n_chains,
                                                        int32_t n_steps, const int32_t* pairs, const double* u,
                                                        int32_t* accepted) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n_chains) return;
  int8_t* xc = x + c * ldx;
  uint64_t mask = load_mask(xc, R.N, lane);
  int32_t acc = 0;
  // with M <= 256 the hidden fields and their logcosh are cached per lane and
  // recomputed only after an accepted move (the configuration changes only then)
  const bool cached = R.M <= 64 * kHPerLane;
  dv2 tc[kHPerLane], lc[kHPerLane];
  auto refresh = [&]() {
#pragma unroll
    for (int q = 0; q < kHPerLane; ++q) {
      const int h = lane + 64 * q;
      if (h < R.M) {
        tc[q] = hidden_field(R, mask, h);
        lc[q] = vlogcosh(tc[q]);
      }
    }
  };
  if (cached) refresh();
  for (int s = 0; s < n_steps; ++s) {
    const int64_t e = (int64_t)s * n_chains + c;
    const int i = pairs[2 * e], j = pairs[2 * e + 1];
    if ((unsigned)i >= (unsigned)R.N || (unsigned)j >= (unsigned)R.N) continue;
    if (((mask >> i) & 1) == ((mask >> j) & 1)) continue;
    const dv2 d = cached ? exchange_ratio_log_cached(R, mask, i, j, lane, tc, lc)
                         : exchange_ratio_log(R, mask, i, j, lane);
    if (u[e] < exp(2.0 * d.x)) {
      mask ^= ((uint64_t)1 << i) | ((uint64_t)1 << j);
      ++acc;
      if (cached) refresh();
    }
  }
  if (lane < R.N) xc[lane] = (mask >> lane) & 1 ? 1 : -1;
  if (lane == 0 && accepted) accepted[c] = acc;
}

// One wave per sample: E_loc = J sum_bonds [x_i x_j / 4 + [x_i != x_j]
// psi(x^{ij}) / (2 psi(x))], bonds (i, i + 1) and, when periodic, (N - 1, 0).
__global__ __launch_bounds__(256) void k_rbm_heisenberg_eloc(const RbmArgs R, const int8_t* x, int64_t ldx,
                                                             int64_t n_s, double J, int32_t periodic,
                                                             double2* e_loc) {
  const int lane = threadIdx.x & 63;
  const int64_t smp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (smp >= n_s) return;
  const uint64_t mask = load_mask(x + smp * ldx, R.N, lane);
  const int nb = periodic && R.N > 2 ? R.N : R.N - 1;
  dv2 e = dv2{0.0, 0.0};
  for (int b = 0; b < nb; ++b) {
    const int i = b, j = b + 1 < R.N ? b + 1 : 0;
    e.x += 0.25 * spin(mask, i) * spin(mask, j);
    if (((mask >> i) & 1) != ((mask >> j) & 1)) {
      const dv2 d = exchange_ratio_log(R, mask, i, j, lane);
      double sn, cs;
      sincos(d.y, &sn, &cs);
      const double m = 0.5 * exp(d.x);
      e += dv2{m * cs, m * sn};
    }
  }
  if (lane == 0) ((QGT_GLOBAL dv2*)e_loc)[smp] = J * e;
}

__global__ __launch_bounds__(256) void k_sr_update(double2* theta, const double2* delta, int64_t n, double eta) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  QGT_GLOBAL dv2* t = (QGT_GLOBAL dv2*)theta + k;
  *t = *t - eta * ((const QGT_GLOBAL dv2*)delta)[k];
}

qgt_status rbm_checks(int32_t N, int32_t M, const void* theta, const void* x, int64_t ldx, int64_t n) {
  if (N < 2 || N > 64) return report_error(QGT_ERR_UNSUPPORTED, "n_visible must be in [2, 64]");
  if (M < 1 || M > 65535) return report_error(QGT_ERR_UNSUPPORTED, "n_hidden must be in [1, 65535]");
  if (!theta || !x) return report_error(QGT_ERR_INVALID_ARGUMENT, "theta or x is null");
  if (ldx < N) return report_error(QGT_ERR_INVALID_ARGUMENT, "ldx < n_visible");
  if (n < 1 || n > ((int64_t)1 << 31) - 4) return report_error(QGT_ERR_UNSUPPORTED, "sample count out of range");
  return QGT_OK;
}

}  // namespace
}  // namespace qgt

using namespace qgt;

extern "C" {

qgt_status qgt_rbm_metropolis(int32_t n_visible, int32_t n_hidden, const void* theta, int8_t* x, int64_t ldx,
                              int64_t n_chains, int32_t n_steps, const int32_t* pairs, const double* u,
                              int32_t* accepted, hipStream_t stream) {
  qgt_status st = rbm_checks(n_visible, n_hidden, theta, x, ldx, n_chains);
  if (st != QGT_OK) return st;
  if (n_steps < 0) return report_error(QGT_ERR_INVALID_ARGUMENT, "n_steps < 0");
  if (n_steps > 0 && (!pairs || !u)) return report_error(QGT_ERR_INVALID_ARGUMENT, "pairs or u is null");
  const RbmArgs R{(const double2*)theta, n_visible, n_hidden};
  hipLaunchKernelGGL(k_rbm_metropolis, dim3((unsigned)((n_chains + 3) / 4)), dim3(256), 0, stream, R, x, ldx,
                     n_chains, n_steps, pairs, u, accepted);
  return report_launch("rbm metropolis");
}

qgt_status qgt_rbm_heisenberg_eloc(int32_t n_visible, int32_t n_hidden, const void* theta, const int8_t* x,
                                   int64_t ldx, int64_t n_s, double J, int32_t periodic, void* e_loc,
                                   hipStream_t stream) {
  qgt_status st = rbm_checks(n_visible, n_hidden, theta, x, ldx, n_s);
  if (st != QGT_OK) return st;
  if (!e_loc) return report_error(QGT_ERR_INVALID_ARGUMENT, "e_loc is null");
  const RbmArgs R{(const double2*)theta, n_visible, n_hidden};
  hipLaunchKernelGGL(k_rbm_heisenberg_eloc, dim3((unsigned)((n_s + 3) / 4)), dim3(256), 0, stream, R, x, ldx, n_s,
                     J, periodic, (double2*)e_loc);
  return report_launch("rbm heisenberg local energy");
}

qgt_status qgt_sr_update(void* theta, const void* delta, int64_t n_p, double eta, hipStream_t stream) {
  if (!theta || !delta) return report_error(QGT_ERR_INVALID_ARGUMENT, "theta or delta is null");
  if (n_p < 1 || n_p > ((int64_t)1 << 31) - 1) return report_error(QGT_ERR_UNSUPPORTED, "n_p out of range");
  hipLaunchKernelGGL(k_sr_update, dim3((unsigned)((n_p + 255) / 256)), dim3(256), 0, stream, (double2*)theta,
                     (const double2*)delta, n_p, eta);
  return report_launch("sr update");
}

}  // extern "C"
