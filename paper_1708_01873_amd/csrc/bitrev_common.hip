// Element-size independent kernels of libbitrev: the batched prep kernel
// (validation and work-count scan) and the reference streaming copy.
#include <limits.h>

#include "bitrev_device.hpp"
#include "bitrev_launch.hpp"

namespace bitrev {
namespace {

constexpr int kPrepThreads = 1024;

// Work items of array a for the batched kernel at tile width b: one
// whole-array item when 2^k < 2^(2b) (none in place for n <= 2, the
// identity), else one per tile pair (in place) or per tile (out of place).
// Sets *bad and returns 0 when the array's metadata is inconsistent.
__device__ int64_t batched_work(const int64_t* offsets, const int32_t* log2n, int64_t a,
                                int64_t data_elems, int b, bool oop, bool* bad) {
  const int k = log2n[a];
  const int64_t o0 = offsets[a];
  const int64_t o1 = offsets[a + 1];
  const bool ok = k >= 0 && k <= 40 && o0 >= 0 && o1 >= o0 && (o1 - o0) == (1ll << k) &&
                  o1 <= data_elems && (k < 2 * b || k - 2 * b <= 32);
  if (!ok) {
    *bad = true;
    return 0;
  }
  if (k < 2 * b) return (k <= 1 && !oop) ? 0 : 1;
  return oop ? (int64_t)1 << (k - 2 * b) : (int64_t)pair_count(k - 2 * b);
}

// One workgroup: each thread takes a contiguous run of arrays, the block
// scans the per-thread sums, then each thread writes its run's exclusive
// prefix sums.  ws[0] = rejected arrays, ws[1] = first rejected (or -1),
// ws[2 + a] = first work id of array a, ws[2 + num] = total work.
__global__ __launch_bounds__(kPrepThreads) void k_batched_prep(const int64_t* offsets,
                                                               const int32_t* log2n, int64_t num,
                                                               int64_t data_elems, int b,
                                                               int oop, int64_t* ws) {
  __shared__ int64_t sum_sh[kPrepThreads];
  __shared__ int64_t bad_sh[kPrepThreads];
  __shared__ int64_t first_sh[kPrepThreads];
  const int t = (int)threadIdx.x;
  const int64_t per = (num + kPrepThreads - 1) / kPrepThreads;
  const int64_t a0 = (int64_t)t * per < num ? (int64_t)t * per : num;
  const int64_t a1 = a0 + per < num ? a0 + per : num;
  int64_t sum = 0, nbad = 0, first = LLONG_MAX;
  for (int64_t a = a0; a < a1; ++a) {
    bool bad = false;
    sum += batched_work(offsets, log2n, a, data_elems, b, oop != 0, &bad);
    if (bad) {
      ++nbad;
      if (first == LLONG_MAX) first = a;
    }
  }
  sum_sh[t] = sum;
  bad_sh[t] = nbad;
  first_sh[t] = first;
  __syncthreads();
  for (int d = 1; d < kPrepThreads; d <<= 1) {  // inclusive scan of the sums
    const int64_t v = t >= d ? sum_sh[t - d] : 0;
    __syncthreads();
    sum_sh[t] += v;
    __syncthreads();
  }
  for (int d = kPrepThreads / 2; d > 0; d >>= 1) {  // rejected count and first
    if (t < d) {
      bad_sh[t] += bad_sh[t + d];
      if (first_sh[t + d] < first_sh[t]) first_sh[t] = first_sh[t + d];
    }
    __syncthreads();
  }
  int64_t run = sum_sh[t] - sum;
  for (int64_t a = a0; a < a1; ++a) {
    ws[2 + a] = run;
    bool bad = false;
    run += batched_work(offsets, log2n, a, data_elems, b, oop != 0, &bad);
  }
  if (t == kPrepThreads - 1) ws[2 + num] = sum_sh[t];
  if (t == 0) {
    ws[0] = bad_sh[0];
    ws[1] = first_sh[0] == LLONG_MAX ? -1 : first_sh[0];
  }
}

// Streaming copy, one 16-byte access per thread per iteration, grid
// stride.  With four workgroups per compute unit this was the fastest of the
// copy shapes measured on MI355X (unrolled, blocked and non-temporal forms
// were slower or equal), so it is the honest denominator for the roofline.
template <int H>
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src,
                                                u32x4* __restrict__ dst, uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nvec; i += stride)
    st_hint<H>(dst + i, ld_hint<H>(src + i));
}

__global__ __launch_bounds__(256) void k_copy1(const uint8_t* __restrict__ src,
                                               uint8_t* __restrict__ dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_batched_prep(const BatchedLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL(k_batched_prep, dim3(1), dim3(kPrepThreads), 0, st, a.offsets, a.log2n, a.num,
                     a.data_elems, a.b, a.src != nullptr ? 1 : 0, a.ws);
  return hipGetLastError();
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, uint32_t grid, int hints,
                       hipStream_t st) {
  const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) == 0;
  const uint64_t nvec = vec ? bytes / 16 : 0;
  if (nvec) {
    if (hints == kHintStreamLoads) {
      hipLaunchKernelGGL(k_copy16<kHintStreamLoads>, dim3(grid), dim3(256), 0, st,
                         static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), nvec);
    } else if (hints == kHintStreamStores) {
      hipLaunchKernelGGL(k_copy16<kHintStreamStores>, dim3(grid), dim3(256), 0, st,
                         static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), nvec);
    } else if (hints == kHintStreamWriteThrough) {
      hipLaunchKernelGGL(k_copy16<kHintStreamWriteThrough>, dim3(grid), dim3(256), 0, st,
                         static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), nvec);
    } else {
      hipLaunchKernelGGL(k_copy16<kHintPlain>, dim3(grid), dim3(256), 0, st,
                         static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), nvec);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const uint64_t done = nvec * 16;
  if (done < bytes) {
    hipLaunchKernelGGL(k_copy1, dim3(grid), dim3(256), 0, st,
                       static_cast<const uint8_t*>(src) + done, static_cast<uint8_t*>(dst) + done,
                       (uint64_t)(bytes - done));
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace bitrev
