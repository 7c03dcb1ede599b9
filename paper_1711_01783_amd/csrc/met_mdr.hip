// Multidimensional reconciliation: the front end of the decoder (Results,
// "Information reconciliation for CV-QKD system"; the rotation method of the
// paper's reference on multidimensional reconciliation, used in reverse
// reconciliation, Methods Step 1).
//
// Alice holds Gaussian variables x, Bob y = x + z.  Both cut their strings into
// blocks of d in {1, 2, 4, 8} values, read as elements of the real Cayley-
// Dickson algebra of dimension d (reals, complex numbers, quaternions,
// octonions), where the product of (a, b) and (c, e) is
// (a c - conj(e) b, e a + b conj(c)) and |p q| = |p| |q|.
//
// Bob maps his unit block y' = y / |y| onto the unit vector u = (1 - 2 b) / sqrt(d)
// of his random bits b: the element alpha = u conj(y') satisfies alpha y' = u
// (alternativity: (u conj(y')) y' = u |y'|^2), and left multiplication by a unit
// element is orthogonal.  He publishes alpha and |y|.  Alice forms
// v = alpha x / |x|, a noisy copy of u; since alpha x = |y| u - alpha z, her
// log-likelihood ratio for bit b = 0 against 1 on the virtual binary-input
// channel is 2 |x| |y| v / (sqrt(d) sigma_z^2) = (2 |y| / (sqrt(d) sigma_z^2)) alpha x.
//
// Both kernels are one pass over the data (HBM-bound): a thread takes one
// block of d values, loads it with vector loads, and writes its outputs; the
// algebra is a few dozen multiply-adds per block in registers.
#include <hip/hip_runtime.h>

#include <cmath>

#include "met_internal.h"

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return met::fail(MET_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

namespace met {
namespace {

constexpr int kMdrBlock = 256;

// conj((a, b)) = (conj(a), -b); the reals are their own conjugates.
template <int D>
__device__ __forceinline__ void cd_conj(const float *p, float *o) {
  if constexpr (D == 1) {
    o[0] = p[0];
  } else {
    cd_conj<D / 2>(p, o);
#pragma unroll
    for (int i = D / 2; i < D; ++i) o[i] = -p[i];
  }
}

// Cayley-Dickson product o = p q (o must not alias p or q).
template <int D>
__device__ __forceinline__ void cd_mul(const float *p, const float *q, float *o) {
  if constexpr (D == 1) {
    o[0] = p[0] * q[0];
  } else {
    constexpr int H = D / 2;
    const float *a = p, *b = p + H, *c = q, *e = q + H;
    float ce[H], cc[H], t0[H], t1[H];
    cd_conj<H>(e, ce);
    cd_conj<H>(c, cc);
    cd_mul<H>(a, c, t0);
    cd_mul<H>(ce, b, t1);
#pragma unroll
    for (int i = 0; i < H; ++i) o[i] = t0[i] - t1[i];
    cd_mul<H>(e, a, t0);
    cd_mul<H>(b, cc, t1);
#pragma unroll
    for (int i = 0; i < H; ++i) o[H + i] = t0[i] + t1[i];
  }
}

template <int D>
__device__ __forceinline__ void load_block(const float *src, float *v) {
  if constexpr (D % 4 == 0) {
#pragma unroll
    for (int i = 0; i < D; i += 4) {
      const float4 t = *reinterpret_cast<const float4 *>(src + i);
      v[i] = t.x;
      v[i + 1] = t.y;
      v[i + 2] = t.z;
      v[i + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) v[i] = src[i];
  }
}

template <int D>
__device__ __forceinline__ void store_block(float *dst, const float *v) {
  if constexpr (D % 4 == 0) {
#pragma unroll
    for (int i = 0; i < D; i += 4) *reinterpret_cast<float4 *>(dst + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) dst[i] = v[i];
  }
}

// Bob: alpha = u conj(y / |y|) per block (y / |y| = e_0 when |y| = 0), |y|.
template <int D>
__global__ __launch_bounds__(kMdrBlock) void k_mdr_bob(const float *y, const uint8_t *bits, int64_t n_blocks,
                                                       float *alpha, float *ynorm) {
  const int64_t t = (int64_t)blockIdx.x * kMdrBlock + threadIdx.x;
  if (t >= n_blocks) return;
  float yv[D], u[D], yc[D], a[D];
  load_block<D>(y + t * D, yv);
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < D; ++i) s = fmaf(yv[i], yv[i], s);
  const float nrm = sqrtf(s);
  if (nrm > 0.0f) {
    const float r = 1.0f / nrm;
#pragma unroll
    for (int i = 0; i < D; ++i) yv[i] *= r;
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) yv[i] = i == 0 ? 1.0f : 0.0f;
  }
  const float us = 1.0f / sqrtf((float)D);
  if constexpr (D == 8) {
    const uint64_t w = *reinterpret_cast<const uint64_t *>(bits + t * D);
#pragma unroll
    for (int i = 0; i < D; ++i) u[i] = ((w >> (8 * i)) & 1ull) ? -us : us;
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i) u[i] = (bits[t * D + i] & 1u) ? -us : us;
  }
  cd_conj<D>(yv, yc);
  cd_mul<D>(u, yc, a);
  store_block<D>(alpha + t * D, a);
  ynorm[t] = nrm;
}

// Alice: llr = (2 |y| / (sqrt(d) sigma_z^2)) alpha x per block.
template <int D>
__global__ __launch_bounds__(kMdrBlock) void k_mdr_alice(const float *x, const float *alpha, const float *ynorm,
                                                         float scale, int64_t n_blocks, float *llr) {
  const int64_t t = (int64_t)blockIdx.x * kMdrBlock + threadIdx.x;
  if (t >= n_blocks) return;
  float xv[D], a[D], v[D];
  load_block<D>(x + t * D, xv);
  load_block<D>(alpha + t * D, a);
  cd_mul<D>(a, xv, v);
  const float k = scale * ynorm[t];
#pragma unroll
  for (int i = 0; i < D; ++i) v[i] *= k;
  store_block<D>(llr + t * D, v);
}

int validate_mdr(int64_t B, int64_t N, int32_t d) {
  if (d != 1 && d != 2 && d != 4 && d != 8) return fail(MET_EINVAL, "dimension %d is not 1, 2, 4 or 8", d);
  if (B < 1 || N < 1) return fail(MET_EINVAL, "B = %lld, N = %lld: both must be >= 1", (long long)B, (long long)N);
  if (N % d) return fail(MET_EINVAL, "N = %lld is not a multiple of the dimension %d", (long long)N, d);
  if (B > ((int64_t)1 << 36) / N) return fail(MET_EINVAL, "B x N = %lld x %lld above 2^36", (long long)B, (long long)N);
  return MET_OK;
}

bool misaligned(const void *p, size_t a) { return ((uintptr_t)p & (a - 1)) != 0; }

unsigned grid_of(int64_t n_blocks) { return (unsigned)((n_blocks + kMdrBlock - 1) / kMdrBlock); }

}  // namespace
}  // namespace met

extern "C" int met_mdr_bob(const float *y, const uint8_t *bits, int64_t B, int64_t N, int32_t d, float *alpha,
                           float *ynorm, void *stream) { return met::guarded("met_mdr_bob", [&]() -> int {
  met::clear_error();
  int rc = met::validate_mdr(B, N, d);
  if (rc) return rc;
  if (!y || !bits || !alpha || !ynorm) return met::fail(MET_EINVAL, "met_mdr_bob: NULL buffer");
  if (met::misaligned(y, 16) || met::misaligned(alpha, 16) || met::misaligned(bits, 8) || met::misaligned(ynorm, 4))
    return met::fail(MET_EINVAL, "met_mdr_bob: y and alpha must be 16-byte, bits 8-byte aligned");
  const int64_t nb = B * (N / d);
  const hipStream_t st = (hipStream_t)stream;
  switch (d) {
    case 1: hipLaunchKernelGGL(met::k_mdr_bob<1>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, y, bits, nb, alpha, ynorm); break;
    case 2: hipLaunchKernelGGL(met::k_mdr_bob<2>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, y, bits, nb, alpha, ynorm); break;
    case 4: hipLaunchKernelGGL(met::k_mdr_bob<4>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, y, bits, nb, alpha, ynorm); break;
    default: hipLaunchKernelGGL(met::k_mdr_bob<8>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, y, bits, nb, alpha, ynorm); break;
  }
  HIP_TRY(hipGetLastError());
  return MET_OK;
  });
}

extern "C" int met_mdr_alice(const float *x, const float *alpha, const float *ynorm, float sigma_z2, int64_t B,
                             int64_t N, int32_t d, float *llr, void *stream) { return met::guarded("met_mdr_alice", [&]() -> int {
  met::clear_error();
  int rc = met::validate_mdr(B, N, d);
  if (rc) return rc;
  if (!x || !alpha || !ynorm || !llr) return met::fail(MET_EINVAL, "met_mdr_alice: NULL buffer");
  if (!(sigma_z2 > 0.0f) || !std::isfinite(sigma_z2))
    return met::fail(MET_EINVAL, "met_mdr_alice: noise variance %g must be positive and finite", (double)sigma_z2);
  if (met::misaligned(x, 16) || met::misaligned(alpha, 16) || met::misaligned(llr, 16) || met::misaligned(ynorm, 4))
    return met::fail(MET_EINVAL, "met_mdr_alice: x, alpha and llr must be 16-byte aligned");
  const int64_t nb = B * (N / d);
  const float scale = (float)(2.0 / (std::sqrt((double)d) * (double)sigma_z2));
  const hipStream_t st = (hipStream_t)stream;
  switch (d) {
    case 1: hipLaunchKernelGGL(met::k_mdr_alice<1>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, x, alpha, ynorm, scale, nb, llr); break;
    case 2: hipLaunchKernelGGL(met::k_mdr_alice<2>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, x, alpha, ynorm, scale, nb, llr); break;
    case 4: hipLaunchKernelGGL(met::k_mdr_alice<4>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, x, alpha, ynorm, scale, nb, llr); break;
    default: hipLaunchKernelGGL(met::k_mdr_alice<8>, dim3(met::grid_of(nb)), dim3(met::kMdrBlock), 0, st, x, alpha, ynorm, scale, nb, llr); break;
  }
  HIP_TRY(hipGetLastError());
  return MET_OK;
  });
}
