// Host-side interface between the C ABI (bitrev_api.hip) and the kernels.
// One translation unit per element size instantiates the kernels for that
// size (bitrev_s<S>.hip) and defines the launchers declared here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bitrev {

constexpr int kMaxTileBits = 7;

// Largest tile width b compiled for element size s.
constexpr int max_tile_bits(int s) { return s >= 8 ? 6 : 7; }

// Smallest tile width the batched kernel is compiled for.
constexpr int kMinBatchedTileBits = 2;

struct TileLaunch {
  const void* src;          // source array(s)
  void* dst;                // destination array(s); == src for in place
  int m;                    // middle bits: log2n - 2b
  uint64_t items_per_seg;   // work items per array
  uint64_t total_items;     // items_per_seg * number of arrays
  uint64_t seg_elems;       // elements between consecutive source arrays (>= 2^log2n)
  uint64_t dst_seg_elems = 0; // between destination arrays (out of place)
  int balanced;             // work-item order: 0 natural, 1 balanced bit dealing
  int xcds;                 // number of XCDs the grid is dealt over
  uint32_t grid;            // workgroups (multiple of xcds)
  int pipelined;            // 1: persistent software-pipelined, 2: register-staged (in place)
  int hints = 0;            // CacheHint of the one-item 16-byte kernels
  void* ev_start = nullptr; // hipEvent_t recorded as the kernel starts (or null)
  void* ev_stop = nullptr;  // hipEvent_t recorded as it ends
};

struct WaveLaunch {
  const void* src;
  void* dst;
  int k;                    // log2n <= 6
  uint64_t nseg;            // number of arrays
  uint32_t grid;
  uint64_t src_stride = 0;  // elements between consecutive arrays
  uint64_t dst_stride = 0;
};

struct DitLaunch {
  TileLaunch t;             // the tile geometry (src == dst: in place)
  int stages;               // DIT levels fused after the reversal, <= b
  int inverse;              // 1: exp(+2 pi i ...) twiddles
  int rect_bz = 0;          // > 0: out of place with rectangular tiles of
                            // 2^b source rows of 2^rect_bz elements
  int rs = 0;               // 1: in place, complex64, the pair held in
                            // registers and staged through one LDS tile
};

struct TransposeLaunch {
  void* data;
  int h;                    // the matrix is 2^h x 2^h elements
  uint64_t total_items;     // tile pairs (R <= C)
  int xcds;
  uint32_t grid;
};

struct BatchedLaunch {
  const void* src = nullptr;  // out of place: the source (data is the destination)
  void* data;
  const int64_t* offsets;
  const int32_t* log2n;
  int64_t num;
  int64_t data_elems;
  int64_t* ws;              // [0] invalid count, [1] first invalid, [2..] scan
  int b;
  int balanced;
  int xcds;
  uint32_t grid;
};

// Threads per workgroup of the tile kernels for (s, b, vec); 0 if not built.
int tile_block_threads(int s, int b, bool vec);
// Threads per workgroup of the batched kernel for (s, b).
int batched_block_threads(int s, int b);
// Static LDS bytes per workgroup of each kernel (for occupancy estimates).
size_t tile_lds_bytes(int s, int b, bool inplace);

#define BITREV_DECLARE_LAUNCHERS(S)                                                  \
  hipError_t launch_tile_inplace_s##S(int b, bool vec, const TileLaunch& a,          \
                                      hipStream_t st);                               \
  hipError_t launch_tile_outofplace_s##S(int b, bool vec, const TileLaunch& a,       \
                                         hipStream_t st);                            \
  hipError_t launch_wave_s##S(const WaveLaunch& a, hipStream_t st);                  \
  hipError_t launch_batched_s##S(const BatchedLaunch& a, hipStream_t st);            \
  hipError_t launch_tile_copy_s##S(int b, const TileLaunch& a, hipStream_t st);      \
  hipError_t launch_block_recursive_s##S(void* data, int h, uint64_t nblocks,        \
                                         bool vec, uint32_t grid, hipStream_t st);   \
  hipError_t launch_transpose_s##S(int b, bool vec, const TransposeLaunch& a,        \
                                   hipStream_t st);                                  \
  hipError_t launch_digit_s##S(int d, int b, bool vec, const TileLaunch& a,          \
                               hipStream_t st);                                      \
  hipError_t launch_wave_digit_s##S(const WaveLaunch& a, int d, hipStream_t st);     \
  hipError_t launch_evenodd_s##S(const void* src, void* dst, int k, uint64_t rows,   \
                                 uint32_t grid, hipStream_t st);                     \
  int tile_threads_s##S(int b, bool vec);                                            \
  int tile_rs_threads_s##S(int b, bool vec);                                         \
  int tile_occupancy_s##S(int b, bool vec, bool inplace, bool pipelined);            \
  int batched_occupancy_s##S(int b, bool oop);                                     \
  int batched_threads_s##S(int b);

BITREV_DECLARE_LAUNCHERS(1)
BITREV_DECLARE_LAUNCHERS(2)
BITREV_DECLARE_LAUNCHERS(4)
BITREV_DECLARE_LAUNCHERS(8)
BITREV_DECLARE_LAUNCHERS(16)

hipError_t launch_dit_s8(int b, bool vec, const DitLaunch& a, hipStream_t st);
hipError_t launch_dit_s16(int b, bool vec, const DitLaunch& a, hipStream_t st);

hipError_t launch_batched_prep(const BatchedLaunch& a, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, uint32_t grid, int hints,
                       hipStream_t st);

}  // namespace bitrev
