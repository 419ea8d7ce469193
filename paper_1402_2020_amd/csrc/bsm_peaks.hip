// Measured rooflines (include/bsm_peaks.h): kernels that do nothing but
// 32-bit integer vector arithmetic, int8 matrix products or streaming HBM
// traffic, timed with HIP events on a private stream.
#include "bsm_peaks.h"

#include <algorithm>

#include "bsm_internal.h"

namespace bsm {
namespace {

typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v16i32 __attribute__((ext_vector_type(16)));
typedef int v8i32 __attribute__((ext_vector_type(8)));
typedef float v16f32 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kValuIters = 4096;
constexpr int kValuPerIter = 32;   // instructions per loop iteration, per lane
constexpr int kMfmaIters = 2048;
constexpr int kMfmaChains = 4;     // independent accumulators per wave
constexpr double kMfmaOps = 32.0 * 32.0 * 32.0 * 2.0;
constexpr double kMfmaFp4Ops = 32.0 * 32.0 * 64.0 * 2.0;

// Four independent chains, 32 instructions per iteration written out in
// assembly so that none is folded or removed.  MIX: the kinds the describe
// and cost kernels issue most (byte permute, bit count, funnel shift, packed
// 16-bit subtract, masked byte SAD, max, and-or, three-input bit operation);
// otherwise alternating adds and xors, which issue faster on gfx950.
#define BSM_PEAK_ADDXOR(j) "v_add_u32 %" #j ", %" #j ", %4\n\tv_xor_b32 %" #j ", %" #j ", %4\n\t"
#define BSM_PEAK_MIX_A(j) \
  "v_perm_b32 %" #j ", %" #j ", %4, %5\n\tv_bcnt_u32_b32 %" #j ", %" #j ", %4\n\t"
#define BSM_PEAK_MIX_B(j) \
  "v_alignbit_b32 %" #j ", %" #j ", %4, 31\n\tv_pk_sub_u16 %" #j ", %" #j ", %4\n\t"
#define BSM_PEAK_MIX_C(j) \
  "v_msad_u8 %" #j ", %" #j ", %4, %" #j "\n\tv_max_u32 %" #j ", %" #j ", %4\n\t"
#define BSM_PEAK_MIX_D(j) \
  "v_and_or_b32 %" #j ", %" #j ", %4, %5\n\tv_bitop3_b32 %" #j ", %" #j ", %4, %5 bitop3:0x1e\n\t"
#define BSM_PEAK_ALL(M) M(0) M(1) M(2) M(3)
template <bool MIX>
__global__ __launch_bounds__(kThreads) void k_peak_valu(uint32_t seed, int iters,
                                                        uint32_t *__restrict__ out) {
  const uint32_t gid = blockIdx.x * kThreads + threadIdx.x;
  uint32_t a = seed ^ gid, b = a * 3u + 1u, c = a * 5u + 7u, d = a * 9u + 3u;
  const uint32_t k = seed | 1u, k2 = seed ^ 0x0c0c0404u;
  for (int i = 0; i < iters; ++i) {
    if constexpr (MIX)
      asm volatile(BSM_PEAK_ALL(BSM_PEAK_MIX_A) BSM_PEAK_ALL(BSM_PEAK_MIX_B)
                       BSM_PEAK_ALL(BSM_PEAK_MIX_C) BSM_PEAK_ALL(BSM_PEAK_MIX_D)
                   : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
                   : "v"(k), "v"(k2));
    else
      asm volatile(BSM_PEAK_ALL(BSM_PEAK_ADDXOR) BSM_PEAK_ALL(BSM_PEAK_ADDXOR)
                       BSM_PEAK_ALL(BSM_PEAK_ADDXOR) BSM_PEAK_ALL(BSM_PEAK_ADDXOR)
                   : "+v"(a), "+v"(b), "+v"(c), "+v"(d)
                   : "v"(k), "v"(k2));
  }
  out[gid] = a ^ b ^ c ^ d;
}
#undef BSM_PEAK_ALL
#undef BSM_PEAK_MIX_D
#undef BSM_PEAK_MIX_C
#undef BSM_PEAK_MIX_B
#undef BSM_PEAK_MIX_A
#undef BSM_PEAK_ADDXOR

__global__ __launch_bounds__(kThreads) void k_peak_mfma(int seed, int iters,
                                                        int *__restrict__ out) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const v4i32 a = {seed ^ gid, gid, seed, 0x01010101};
  const v4i32 b = {gid * 3, seed ^ 0x5a5a5a5a, 0x7f7f7f7f, gid};
  v16i32 acc[kMfmaChains];
#pragma unroll
  for (int j = 0; j < kMfmaChains; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = j + e;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kMfmaChains; ++j)
      acc[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[j], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int j = 0; j < kMfmaChains; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  out[gid] = s;
}

// The same with v_mfma_scale_f32_32x32x64_f8f6f4 on e2m1 (fp4) operands at
// unit scale (E8M0 127), the product the matrix-core cost kernels issue;
// operands use the low four dwords.
__global__ __launch_bounds__(kThreads) void k_peak_mfma_fp4(int seed, int iters,
                                                            int *__restrict__ out) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const v8i32 a = {seed ^ gid, gid, seed, 0x22222222, 0, 0, 0, 0};
  const v8i32 b = {gid * 3, seed ^ 0x15151515, 0x21212121, gid, 0, 0, 0, 0};
  v16f32 acc[kMfmaChains];
#pragma unroll
  for (int j = 0; j < kMfmaChains; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = static_cast<float>(j + e);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kMfmaChains; ++j)
      acc[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[j], 4, 4, 0, 127, 0, 127);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < kMfmaChains; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  out[gid] = static_cast<int>(s);
}

// Grid-stride streaming read, four 16-byte loads in flight per lane.
__global__ __launch_bounds__(kThreads) void k_peak_read(const uint4 *__restrict__ p, size_t n16,
                                                        uint32_t *__restrict__ out) {
  const size_t gid = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * kThreads;
  uint32_t x = 0;
  size_t i = gid;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 v0 = p[i], v1 = p[i + stride], v2 = p[i + 2 * stride], v3 = p[i + 3 * stride];
    x ^= v0.x ^ v0.y ^ v0.z ^ v0.w ^ v1.x ^ v1.y ^ v1.z ^ v1.w;
    x ^= v2.x ^ v2.y ^ v2.z ^ v2.w ^ v3.x ^ v3.y ^ v3.z ^ v3.w;
  }
  for (; i < n16; i += stride) {
    const uint4 v = p[i];
    x ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  out[gid] = x;
}

__global__ __launch_bounds__(kThreads) void k_peak_copy(const uint4 *__restrict__ src,
                                                        uint4 *__restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride],
                v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

// Owns the probe's device memory, events and stream; releases them in reverse.
struct Probe {
  void *buf = nullptr, *out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Probe() {
    if (s) (void)hipStreamSynchronize(s);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    if (buf) (void)hipFree(buf);
  }
};

}  // namespace
}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_measure_peaks(int device, size_t hbm_bytes, int reps, bsm_peaks *out) {
  clear_error();
  if (!out) return fail(BSM_EINVAL, "peaks output is NULL");
  if (reps < 1) return fail(BSM_EINVAL, "reps %d must be >= 1", reps);
  if (hbm_bytes < (size_t(256) << 20) || hbm_bytes % (size_t(64) << 10))
    return fail(BSM_EINVAL, "hbm_bytes %zu must be a multiple of 64 KiB and >= 256 MiB", hbm_bytes);
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return fail(BSM_EINVAL, "device %d out of [0, %d)", device, count);
  DeviceGuard guard(device);
  if (guard.err() != hipSuccess) return fail(BSM_EDEVICE, "hipSetDevice: %s", hipGetErrorString(guard.err()));
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(BSM_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  const int cus = prop.multiProcessorCount;
  const int valu_blocks = cus * 8, mfma_blocks = cus * 4, mem_blocks = cus * 8;
  const size_t out_bytes = (size_t)valu_blocks * kThreads * sizeof(uint32_t);

  Probe p;
  if (hipMalloc(&p.buf, hbm_bytes) != hipSuccess || hipMalloc(&p.out, out_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BSM_ENOMEM, "cannot allocate %zu bytes for the probes", hbm_bytes + out_bytes);
  }
  if ((e = hipStreamCreate(&p.s)) != hipSuccess || (e = hipEventCreate(&p.e0)) != hipSuccess ||
      (e = hipEventCreate(&p.e1)) != hipSuccess ||
      (e = hipMemsetAsync(p.buf, 0x5b, hbm_bytes, p.s)) != hipSuccess)
    return fail(BSM_EDEVICE, "probe set-up: %s", hipGetErrorString(e));

  // Best time in ms of `reps` timed launches after one untimed launch.
  auto best_ms = [&](auto launch, float *ms) -> hipError_t {
    launch();
    *ms = 1e30f;
    for (int r = 0; r < reps; ++r) {
      hipError_t err;
      if ((err = hipEventRecord(p.e0, p.s)) != hipSuccess) return err;
      launch();
      if ((err = hipGetLastError()) != hipSuccess) return err;
      if ((err = hipEventRecord(p.e1, p.s)) != hipSuccess) return err;
      if ((err = hipEventSynchronize(p.e1)) != hipSuccess) return err;
      float t = 0.f;
      if ((err = hipEventElapsedTime(&t, p.e0, p.e1)) != hipSuccess) return err;
      *ms = std::min(*ms, t);
    }
    return hipSuccess;
  };

  const size_t n16 = hbm_bytes / 16, half16 = n16 / 2;
  const uint4 *src = static_cast<const uint4 *>(p.buf);
  uint4 *dst = static_cast<uint4 *>(p.buf) + half16;
  float t_valu, t_addxor, t_mfma, t_fp4, t_read, t_copy;
  if ((e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_valu<true>, dim3(valu_blocks), dim3(kThreads), 0, p.s,
                            0x9e3779b9u, kValuIters, static_cast<uint32_t *>(p.out));
       }, &t_valu)) != hipSuccess ||
      (e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_valu<false>, dim3(valu_blocks), dim3(kThreads), 0, p.s,
                            0x9e3779b9u, kValuIters, static_cast<uint32_t *>(p.out));
       }, &t_addxor)) != hipSuccess ||
      (e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_mfma, dim3(mfma_blocks), dim3(kThreads), 0, p.s, 0x1402,
                            kMfmaIters, static_cast<int *>(p.out));
       }, &t_mfma)) != hipSuccess ||
      (e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_mfma_fp4, dim3(mfma_blocks), dim3(kThreads), 0, p.s, 0x1402,
                            kMfmaIters, static_cast<int *>(p.out));
       }, &t_fp4)) != hipSuccess ||
      (e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_read, dim3(mem_blocks), dim3(kThreads), 0, p.s, src, n16,
                            static_cast<uint32_t *>(p.out));
       }, &t_read)) != hipSuccess ||
      (e = best_ms([&] {
         hipLaunchKernelGGL(k_peak_copy, dim3(mem_blocks), dim3(kThreads), 0, p.s, src, dst,
                            half16);
       }, &t_copy)) != hipSuccess)
    return fail(BSM_EDEVICE, "probe launch: %s", hipGetErrorString(e));

  const double valu_lane_ops = (double)valu_blocks * kThreads * kValuIters * kValuPerIter;
  const double mfma_ops = (double)mfma_blocks * (kThreads / 64) * kMfmaIters * kMfmaChains * kMfmaOps;
  out->valu_int32_ops = valu_lane_ops / (t_valu * 1e-3);
  out->valu_addxor_ops = valu_lane_ops / (t_addxor * 1e-3);
  out->mfma_i8_ops = mfma_ops / (t_mfma * 1e-3);
  out->mfma_fp4_ops = mfma_ops / kMfmaOps * kMfmaFp4Ops / (t_fp4 * 1e-3);
  out->hbm_read_bps = (double)n16 * 16 / (t_read * 1e-3);
  out->hbm_copy_bps = (double)half16 * 16 * 2 / (t_copy * 1e-3);
  out->compute_units = cus;
  return BSM_OK;
}
