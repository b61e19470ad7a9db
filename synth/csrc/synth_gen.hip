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
  const double rho = sqrt(-2.0 * log(u1));
  const double ang = (2.0 * M_PI) * u2;
  double* o = out + (size_t)blockIdx.y * entries;
  const int64_t e0 = 2 * p;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t e = e0 + h;
    if (e < entries) {
      double v = sigma * (h ? rho * sin(ang) : rho * cos(ang));
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
