// Device-side seeded input generator (no solver arithmetic).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with the same counter
// layout, 53-bit uniform construction and Box-Muller transform as the host
// generator in synth/philox.py:
//   counter = (lo32(e >> 1), hi32(e >> 1), stream, tag), key = 64-bit seed
//   m1 = (x0 >> 5) 2^26 + (x1 >> 6), u1 = (m1 + 1) 2^-53 in (0, 1]
//   m2 = (x2 >> 5) 2^26 + (x3 >> 6), u2 = m2 2^-53 in [0, 1)
//   z(e) = sqrt(-2 ln u1) * (e even ? cos : sin)(2 pi u2)
// value = sigma * z + diag * [row == col].
// ln, cos and sin are the generator's own series (ln_unit, cos_sin_turns),
// the same operations in the same order as the host's, on the same nearest
// doubles; the file is built with -ffp-contract=off, so no multiply-add is
// fused and every value equals the host's bit for bit (sqrt and division
// are correctly rounded on both sides).
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace {

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

constexpr double LN2 = 0x1.62e42fefa39efp-1;        // nearest double to ln 2
constexpr double HALF_PI = 0x1.921fb54442d18p+0;   // nearest double to pi / 2
constexpr double SQRT_HALF = 0x1.6a09e667f3bcdp-1;  // nearest double to sqrt(1/2)
// nearest doubles to 1 / (2k + 1), k = 0..11
__constant__ const double LOG_COEF[12] = {
    0x1.0000000000000p+0, 0x1.5555555555555p-2, 0x1.999999999999ap-3, 0x1.2492492492492p-3,
    0x1.c71c71c71c71cp-4, 0x1.745d1745d1746p-4, 0x1.3b13b13b13b14p-4, 0x1.1111111111111p-4,
    0x1.e1e1e1e1e1e1ep-5, 0x1.af286bca1af28p-5, 0x1.8618618618618p-5, 0x1.642c8590b2164p-5};
// nearest doubles to (-1)^k / (2k + 1)!, k = 0..9
__constant__ const double SIN_COEF[10] = {
    0x1.0000000000000p+0, -0x1.5555555555555p-3, 0x1.1111111111111p-7, -0x1.a01a01a01a01ap-13,
    0x1.71de3a556c734p-19, -0x1.ae64567f544e4p-26, 0x1.6124613a86d09p-33, -0x1.ae7f3e733b81fp-41,
    0x1.952c77030ad4ap-49, -0x1.2f49b46814157p-57};
// nearest doubles to (-1)^k / (2k)!, k = 0..10
__constant__ const double COS_COEF[11] = {
    0x1.0000000000000p+0, -0x1.0000000000000p-1, 0x1.5555555555555p-5, -0x1.6c16c16c16c17p-10,
    0x1.a01a01a01a01ap-16, -0x1.27e4fb7789f5cp-22, 0x1.1eed8eff8d898p-29, -0x1.93974a8c07c9dp-37,
    0x1.ae7f3e733b81fp-45, -0x1.6827863b97d97p-53, 0x1.e542ba4020225p-62};

// ln u for u in (0, 1]: u = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// ln m = 2 artanh(s) = 2 s sum_k s^(2k) / (2k + 1), s = (m - 1) / (m + 1).
__device__ inline double ln_unit(double u) {
  int e;
  double m = frexp(u, &e);
  if (m < SQRT_HALF) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = LOG_COEF[11];
#pragma unroll
  for (int k = 10; k >= 0; --k) p = p * z + LOG_COEF[k];
  const double t = s * p;
  return (double)e * LN2 + (t + t);
}

// (cos 2 pi u, sin 2 pi u) for u in [0, 1): 4u = q + r (q the nearest
// integer), theta = r pi / 2 in [-pi/4, pi/4], Taylor series in theta, then
// the quadrant q mod 4 rotates the pair.
__device__ inline void cos_sin_turns(double u, double* c, double* s) {
  const double w = 4.0 * u;
  const double q = floor(w + 0.5);
  const double th = (w - q) * HALF_PI;
  const double x2 = th * th;
  double ps = SIN_COEF[9];
#pragma unroll
  for (int k = 8; k >= 0; --k) ps = ps * x2 + SIN_COEF[k];
  double pc = COS_COEF[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) pc = pc * x2 + COS_COEF[k];
  const double sn = th * ps;
  switch ((int)q & 3) {
    case 0: *c = pc; *s = sn; break;
    case 1: *c = -sn; *s = pc; break;
    case 2: *c = -pc; *s = -sn; break;
    default: *c = sn; *s = -pc; break;
  }
}

// Each thread produces the two normals of one Philox call (entries 2p, 2p+1).
__global__ void gen_matrix_kernel(double* out, int64_t rows, int64_t cols, uint32_t stream0, uint32_t tag,
                                  uint64_t seed, double diag, double sigma) {
  const int64_t entries = rows * cols;
  const int64_t pairs = (entries + 1) / 2;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= pairs) return;
  const uint32_t stream = stream0 + blockIdx.y;
  uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), stream, tag};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t m1 = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);
  const uint64_t m2 = ((uint64_t)(c[2] >> 5) << 26) | (uint64_t)(c[3] >> 6);
  const double u1 = ((double)m1 + 1.0) * 0x1p-53;
  const double u2 = (double)m2 * 0x1p-53;
  const double rho = sqrt(-2.0 * ln_unit(u1));
  double cs, sn;
  cos_sin_turns(u2, &cs, &sn);
  double* o = out + (size_t)blockIdx.y * entries;
  const int64_t e0 = 2 * p;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t e = e0 + h;
    if (e < entries) {
      double v = sigma * (h ? rho * sn : rho * cs);
      if (diag != 0.0 && (e / cols) == (e % cols)) v += diag;
      o[e] = v;
    }
  }
}

__global__ void philox_kernel(uint32_t* out, int64_t count, const uint32_t* ctr, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

}  // namespace

extern "C" {

// out[e][rows][cols] for streams stream0 + e, e < n_stream (device pointer).
int synth_gen_matrix(double* out, int64_t rows, int64_t cols, int32_t n_stream, uint32_t stream0, uint32_t tag,
                     uint64_t seed, double diag, double sigma, hipStream_t stream) {
  if (!out || rows <= 0 || cols <= 0 || n_stream <= 0 || n_stream > 65535) return -1;
  const int64_t pairs = (rows * cols + 1) / 2;
  const int64_t blocks = (pairs + 255) / 256;
  if (blocks > 0x7fffffff) return -1;
  hipLaunchKernelGGL(gen_matrix_kernel, dim3((unsigned)blocks, (unsigned)n_stream), dim3(256), 0, stream, out, rows,
                     cols, stream0, tag, seed, diag, sigma);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

// Raw Philox4x32-10 outputs for count counters (device pointers, 4 words each).
int synth_philox(uint32_t* out, int64_t count, const uint32_t* ctr, uint64_t seed, hipStream_t stream) {
  if (!out || !ctr || count <= 0) return -1;
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, out, count, ctr, seed);
  return hipGetLastError() == hipSuccess ? 0 : -6;
}

}
