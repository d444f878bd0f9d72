// Kernels of libbitrev, instantiated for one element size BITREV_S per
// translation unit (bitrev_s<S>.hip includes this file).
#include <hip/hip_ext.h>

#include "bitrev_device.hpp"
#include "bitrev_launch.hpp"

#ifndef BITREV_S
#error "define BITREV_S (element size in bytes) before including bitrev_kernels.inl"
#endif

namespace bitrev {
namespace {

// Launch `kernel`; non-null events are recorded by the dispatch itself as
// the kernel starts and ends, so that they time the kernel alone.
template <typename F, typename... Args>
hipError_t launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t st, void* ev_start,
                        void* ev_stop, Args... args) {
  hipExtLaunchKernelGGL(kernel, grid, block, 0, st, static_cast<hipEvent_t>(ev_start),
                        static_cast<hipEvent_t>(ev_stop), 0, args...);
  return hipGetLastError();
}

// In place, one array or `total_items / items_per_seg` equal arrays: work
// item -> (array, pair y <= rev_m(y)) -> swap the two tiles through LDS.
template <int S, int B, bool VEC, int H>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_inplace(
    void* data, int m, uint64_t items_per_seg, uint64_t total_items, uint64_t seg_elems,
    int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = tile_threads<S, B, VEC>();
  __shared__ E lds[2 * TileShape<S, B, VEC>::TILE_E];
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    const uint32_t y = inplace_pair_at(m, local, balanced);
    tile_pair_inplace<S, B, VEC, NT, H>(static_cast<E*>(data) + seg * seg_elems, m, y, lds);
    __syncthreads();
  }
}

// In place, register-staged: as k_tile_inplace, with the pair held in
// registers and transposed through a single LDS tile by half as many
// threads (see tile_pair_inplace_rs).
template <int S, int B, bool VEC, int H>
__global__ __launch_bounds__((rs_threads<S, B, VEC>())) void k_tile_inplace_rs(
    void* data, int m, uint64_t items_per_seg, uint64_t total_items, uint64_t seg_elems,
    int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = rs_threads<S, B, VEC>();
  __shared__ E lds[TileShape<S, B, VEC>::TILE_E];
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    const uint32_t y = inplace_pair_at(m, local, balanced);
    tile_pair_inplace_rs<S, B, VEC, NT, H>(static_cast<E*>(data) + seg * seg_elems, m, y, lds);
    __syncthreads();
  }
}

// Out of place: work item -> (array, tile y) -> tile rev_m(y) of dst.
template <int S, int B, bool VEC, int H>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_outofplace(
    const void* src, void* dst, int m, uint64_t items_per_seg, uint64_t total_items,
    uint64_t seg_elems, uint64_t dst_seg_elems, int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = tile_threads<S, B, VEC>();
  __shared__ E lds[TileShape<S, B, VEC>::TILE_E];
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    const uint32_t y = oop_tile_at(m, (uint32_t)local, balanced);
    tile_outofplace<S, B, VEC, NT, H>(static_cast<const E*>(src) + seg * seg_elems,
                                      static_cast<E*>(dst) + seg * dst_seg_elems, m, y, lds);
    __syncthreads();
  }
}

// A copy in the out-of-place tile kernels' order (the identity map in
// place of the reversal): work item -> tile y; its 2^b rows of src are
// written to the same places of dst.  Same reads, same row shape on the
// write side, no LDS stage: the reference copy for the tile kernels where a
// linear sweep is not the fastest way through memory.
template <int S, int B, int H>
__global__ __launch_bounds__((tile_threads<S, B, true>())) void k_tile_copy(
    const void* src, void* dst, int m, uint64_t total_items, int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, true> Sh;
  typedef typename Bytes<Sh::VB>::T V;
  constexpr int NT = tile_threads<S, B, true>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  const uint64_t rowstride = 1ull << (m + B);
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    const uint32_t y = oop_tile_at(m, (uint32_t)item, balanced);
    Chunk<S, Sh::VB> r[PT];
    tile_load<S, B, true, NT, PT, H>(r, static_cast<const E*>(src), rowstride, y);
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int q = (int)threadIdx.x + i * NT;
      if (Sh::CPT % NT == 0 || q < Sh::CPT) {
        const int x = q / Sh::CPR;
        const int zc = q % Sh::CPR;
        const uint64_t off =
            (uint64_t)x * rowstride + (uint64_t)y * Sh::R + (uint64_t)(zc * Sh::CE);
        st_hint<H>(reinterpret_cast<V*>(static_cast<E*>(dst) + off), r[i].v);
      }
    }
  }
}

// Where work item `item` lives: its array's base and its middle bits.
template <typename E>
__device__ __forceinline__ E* item_base(void* data, uint64_t item, uint64_t items_per_seg,
                                        uint64_t total_items, uint64_t seg_elems, uint64_t* local) {
  uint64_t seg = 0;
  *local = item;
  if (items_per_seg != total_items) {
    seg = item / items_per_seg;
    *local = item - seg * items_per_seg;
  }
  return static_cast<E*>(data) + seg * seg_elems;
}

// In place, persistent and software-pipelined: each workgroup walks its work
// items with a grid stride and issues the global loads of the next tile pair
// before it writes out the current one, so that every workgroup keeps reads
// and writes in flight together.  The register copy of the next pair is
// taken only after the current pair sits in LDS.
template <int S, int B, bool VEC>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_inplace_pipe(
    void* data, int m, uint64_t items_per_seg, uint64_t total_items, uint64_t seg_elems,
    int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, VEC> Sh;
  constexpr int NT = tile_threads<S, B, VEC>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  __shared__ E lds[2 * Sh::TILE_E];
  const uint64_t rowstride = 1ull << (m + B);
  Chunk<S, Sh::VB> ra[PT], rb[PT];
  uint64_t item = xcd_block(xcds);
  if (item >= total_items) return;
  uint64_t local;
  E* base = item_base<E>(data, item, items_per_seg, total_items, seg_elems, &local);
  uint32_t y = inplace_pair_at(m, local, balanced);
  uint32_t yr = rev_bits(y, m);
  tile_load<S, B, VEC, NT, PT>(ra, base, rowstride, y);
  if (yr != y) tile_load<S, B, VEC, NT, PT>(rb, base, rowstride, yr);
  while (true) {
    rev_scatter<S, B, VEC, NT, PT>(ra, lds);
    if (yr != y) rev_scatter<S, B, VEC, NT, PT>(rb, lds + Sh::TILE_E);
    __syncthreads();
    const uint64_t next = item + gridDim.x;
    E* nbase = base;
    uint32_t ny = 0, nyr = 0;
    if (next < total_items) {
      nbase = item_base<E>(data, next, items_per_seg, total_items, seg_elems, &local);
      ny = inplace_pair_at(m, local, balanced);
      nyr = rev_bits(ny, m);
      tile_load<S, B, VEC, NT, PT>(ra, nbase, rowstride, ny);
      if (nyr != ny) tile_load<S, B, VEC, NT, PT>(rb, nbase, rowstride, nyr);
    }
    if (yr != y) rev_store<S, B, VEC, NT, PT>(base, rowstride, y, lds + Sh::TILE_E);
    rev_store<S, B, VEC, NT, PT>(base, rowstride, yr, lds);
    if (next >= total_items) break;
    __syncthreads();
    item = next;
    base = nbase;
    y = ny;
    yr = nyr;
  }
}

// Out of place, persistent and software-pipelined (see k_tile_inplace_pipe).
template <int S, int B, bool VEC>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_outofplace_pipe(
    const void* src, void* dst, int m, uint64_t items_per_seg, uint64_t total_items,
    uint64_t seg_elems, uint64_t dst_seg_elems, int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, VEC> Sh;
  constexpr int NT = tile_threads<S, B, VEC>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  __shared__ E lds[Sh::TILE_E];
  const uint64_t rowstride = 1ull << (m + B);
  Chunk<S, Sh::VB> ra[PT];
  uint64_t item = xcd_block(xcds);
  if (item >= total_items) return;
  uint64_t local;
  const E* in = item_base<E>(const_cast<void*>(src), item, items_per_seg, total_items, seg_elems, &local);
  E* out = static_cast<E*>(dst) + (uint64_t)(in - static_cast<const E*>(src)) / seg_elems * dst_seg_elems;
  uint32_t y = oop_tile_at(m, (uint32_t)local, balanced);
  tile_load<S, B, VEC, NT, PT>(ra, in, rowstride, y);
  while (true) {
    rev_scatter<S, B, VEC, NT, PT>(ra, lds);
    __syncthreads();
    const uint64_t next = item + gridDim.x;
    const E* nin = in;
    uint32_t ny = 0;
    if (next < total_items) {
      nin = item_base<E>(const_cast<void*>(src), next, items_per_seg, total_items, seg_elems, &local);
      ny = oop_tile_at(m, (uint32_t)local, balanced);
      tile_load<S, B, VEC, NT, PT>(ra, nin, rowstride, ny);
    }
    rev_store<S, B, VEC, NT, PT>(out, rowstride, rev_bits(y, m), lds);
    if (next >= total_items) break;
    __syncthreads();
    item = next;
    in = nin;
    out = static_cast<E*>(dst) + (uint64_t)(in - static_cast<const E*>(src)) / seg_elems * dst_seg_elems;
    y = ny;
  }
}

// In-place transpose of a 2^h x 2^h matrix: work item -> tile pair
// (R <= C) -> swap (R, C) and (C, R) through LDS.
template <int S, int B, bool VEC>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_transpose_inplace(
    void* data, int h, uint64_t total_items, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = tile_threads<S, B, VEC>();
  __shared__ E lds[2 * TileShape<S, B, VEC>::TILE_E];
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint32_t tr, tc;
    tri_pair(item, &tr, &tc);
    tile_pair_transpose<S, B, VEC, NT>(static_cast<E*>(data), h, tr, tc, lds);
    __syncthreads();
  }
}

// The paper's recursive method one level further down (Methods, recursive
// permutation; Results: its GPU variant recurses twice), for the
// block-local reversals of the recursive scheme: each contiguous block of
// 2^h elements (h even) is staged in LDS and reversed there by the same
// three steps the whole array goes through -- reverse the low h/2 bits
// within every run of 2^(h/2) elements, transpose the 2^(h/2) x 2^(h/2)
// square, reverse the low h/2 bits again.  Each step is an involution, done
// by swapping the pairs i < f(i) in LDS between barriers.  Dynamic LDS holds
// one block (2^h * S bytes).
template <int S, bool VEC>
__global__ __launch_bounds__(512) void k_block_recursive(void* data, int h, uint64_t nblocks) {
  typedef typename Bytes<S>::T E;
  extern __shared__ __align__(16) unsigned char block_lds[];
  E* lds = reinterpret_cast<E*>(block_lds);
  const uint32_t n = 1u << h;
  const int q = h >> 1;
  const uint32_t low = (1u << q) - 1u;
  const uint32_t nvec = VEC ? (uint32_t)(((uint64_t)n * S) / 16) : 0u;
  for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    E* base = static_cast<E*>(data) + blk * (uint64_t)n;
    if constexpr (VEC) {
      const u32x4* src = reinterpret_cast<const u32x4*>(base);
      u32x4* l = reinterpret_cast<u32x4*>(block_lds);
      for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) l[v] = src[v];
    } else {
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds[i] = base[i];
    }
    __syncthreads();
    // step 1: [r | c] -> [r | rev(c)]
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t j = (i & ~low) | rev_bits(i & low, q);
      if (i < j) {
        const E t = lds[i];
        lds[i] = lds[j];
        lds[j] = t;
      }
    }
    __syncthreads();
    // step 2: the square transpose, [r | c] -> [c | r]
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t j = ((i & low) << q) | (i >> q);
      if (i < j) {
        const E t = lds[i];
        lds[i] = lds[j];
        lds[j] = t;
      }
    }
    __syncthreads();
    // step 3: [r | c] -> [r | rev(c)] again
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t j = (i & ~low) | rev_bits(i & low, q);
      if (i < j) {
        const E t = lds[i];
        lds[i] = lds[j];
        lds[j] = t;
      }
    }
    __syncthreads();
    if constexpr (VEC) {
      u32x4* dst = reinterpret_cast<u32x4*>(base);
      const u32x4* l = reinterpret_cast<const u32x4*>(block_lds);
      for (uint32_t v = threadIdx.x; v < nvec; v += blockDim.x) dst[v] = l[v];
    } else {
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) base[i] = lds[i];
    }
    __syncthreads();
  }
}

#if BITREV_S == 8 || BITREV_S == 16
// Bit reversal fused with the first `stages` radix-2 DIT levels (complex
// elements), in place (tile pairs) or out of place.  The radix-8 step of
// dit_rows is used for complex64 except in place at b = 6, where it needs
// more than the 64 VGPRs that two 1024-thread workgroups per CU allow (it
// measured 15% slower there at six levels); complex128 (double registers)
// lost occupancy and 2-10% with it at every width, and keeps radix 4.
template <int S, int B, bool INPLACE>
constexpr int dit_max_radix() { return (S == 8 && !(INPLACE && B >= 6)) ? 8 : 4; }

// Tile steps of the register-staged DIT kernel: the strided-row forms where
// the thread count allows them (fewer registers held across the item loop;
// the two-tile kernel measured 1% slower with them at three and five
// levels, and keeps the general forms).
template <int S, int B, bool VEC, int NT, int PT, int H>
__device__ __forceinline__ void dit_load(Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                         const typename Bytes<S>::T* base, uint64_t rowstride,
                                         uint32_t y) {
  if constexpr (tile_rows_strided<S, B, VEC, NT, PT>())
    tile_load_rows<S, B, VEC, NT, PT, H>(reg, base, rowstride, y);
  else
    tile_load<S, B, VEC, NT, PT, H>(reg, base, rowstride, y);
}

template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void dit_scatter(const Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                            typename Bytes<S>::T* lds) {
  if constexpr (tile_rows_strided<S, B, VEC, NT, PT>())
    tile_scatter_rows<S, B, VEC, NT, PT>(reg, lds);
  else
    tile_scatter<S, B, VEC, NT, PT>(reg, lds);
}

template <int S, int B, bool VEC, int NT, int PT, int H>
__device__ __forceinline__ void dit_store(typename Bytes<S>::T* base, uint64_t rowstride,
                                          uint32_t y, const typename Bytes<S>::T* lds) {
  if constexpr (tile_rows_strided<S, B, VEC, NT, PT>())
    tile_store_rows<S, B, VEC, NT, PT, H>(base, rowstride, y, lds);
  else
    tile_store<S, B, VEC, NT, PT, H>(base, rowstride, y, lds);
}

template <int S, int B, bool VEC, bool INPLACE, int H>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_dit(
    const void* src, void* dst, int m, uint64_t items_per_seg, uint64_t total_items,
    uint64_t seg_elems, int stages, int inverse, int order, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, VEC> Sh;
  typedef typename ComplexOf<S>::T F;
  constexpr int NT = tile_threads<S, B, VEC>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  constexpr int PRE = dit_reg_levels_of<Sh::CPT, Sh::CPR, NT>();
  __shared__ E lds[(INPLACE ? 2 : 1) * Sh::TILE_E];
  __shared__ F tw[(1 << B) > 1 ? (1 << B) : 2];
  make_twiddles<S, B, NT>(tw);
  const uint64_t rowstride = 1ull << (m + B);
  constexpr int MAXR = dit_max_radix<S, B, INPLACE>();
  const bool pre = dit_pre_pays(stages, PRE, MAXR);  // levels 1 .. PRE in registers
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    const E* in = static_cast<const E*>(src) + seg * seg_elems;
    E* out = static_cast<E*>(dst) + seg * seg_elems;
    Chunk<S, Sh::VB> ra[PT];
    if constexpr (INPLACE) {
      Chunk<S, Sh::VB> rb[PT];
      const uint32_t y = inplace_pair_at(m, local, order);
      const uint32_t yr = rev_bits(y, m);
      const bool pal = (y == yr);
      tile_load<S, B, VEC, NT, PT, H>(ra, in, rowstride, y);
      if (!pal) tile_load<S, B, VEC, NT, PT, H>(rb, in, rowstride, yr);
      if constexpr (PRE > 0) {
        dit_reg_levels<S, Sh::VB, PT>(ra, pre, inverse != 0);
        if (!pal) dit_reg_levels<S, Sh::VB, PT>(rb, pre, inverse != 0);
      }
      tile_scatter<S, B, VEC, NT, PT>(ra, lds);
      if (!pal) tile_scatter<S, B, VEC, NT, PT>(rb, lds + Sh::TILE_E);
      __syncthreads();
      dit_rows_after<S, B, NT, MAXR, PRE>(lds, pal ? Sh::R : 2 * Sh::R, stages, inverse != 0, tw,
                                          pre);
      if (!pal) tile_store<S, B, VEC, NT, PT, H>(out, rowstride, y, lds + Sh::TILE_E);
      tile_store<S, B, VEC, NT, PT, H>(out, rowstride, yr, lds);
    } else {
      const uint32_t y = oop_tile_at(m, (uint32_t)local, order);
      tile_load<S, B, VEC, NT, PT, H>(ra, in, rowstride, y);
      if constexpr (PRE > 0) dit_reg_levels<S, Sh::VB, PT>(ra, pre, inverse != 0);
      tile_scatter<S, B, VEC, NT, PT>(ra, lds);
      __syncthreads();
      dit_rows_after<S, B, NT, MAXR, PRE>(lds, Sh::R, stages, inverse != 0, tw, pre);
      tile_store<S, B, VEC, NT, PT, H>(out, rowstride, rev_bits(y, m), lds);
    }
    __syncthreads();
  }
}

// Waves per SIMD the register-staged DIT kernel is compiled for: as many as
// the LDS lets workgroups share a compute unit where the registers allow
// (complex64 b = 6: four workgroups of 33.5 KiB; complex128 b = 6: two).
template <int S, int B, bool VEC> constexpr int rs_dit_waves() {
  return S == 16 ? 4 : ((B == 6 && VEC) ? 8 : 6);
}

// In place, register-staged: half the threads of k_tile_dit hold
// the pair in registers; each tile in turn is staged through one LDS tile,
// takes the levels there and is written over its partner.  Both tiles are
// read before either is written, and no other workgroup touches them.  One
// LDS tile per workgroup instead of two lets four workgroups share a compute
// unit at b = 6 instead of two.
template <int S, int B, bool VEC, int H>
__global__ __launch_bounds__((rs_threads<S, B, VEC>()), (rs_dit_waves<S, B, VEC>())) void k_tile_dit_rs(
    void* data, int m, uint64_t items_per_seg, uint64_t total_items, uint64_t seg_elems,
    int stages, int inverse, int order, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, VEC> Sh;
  typedef typename ComplexOf<S>::T F;
  constexpr int NT = rs_threads<S, B, VEC>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  constexpr int PRE = dit_reg_levels_of<Sh::CPT, Sh::CPR, NT>();
  __shared__ E lds[Sh::TILE_E];
  __shared__ F tw[(1 << B) > 1 ? (1 << B) : 2];
  make_twiddles<S, B, NT>(tw);
  const uint64_t rowstride = 1ull << (m + B);
  const bool pre = dit_pre_pays(stages, PRE, 4);  // levels 1 .. PRE in registers
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    E* base = static_cast<E*>(data) + seg * seg_elems;
    const uint32_t y = inplace_pair_at(m, local, order);
    const uint32_t yr = rev_bits(y, m);
    const bool pal = (y == yr);
    Chunk<S, Sh::VB> ra[PT], rb[PT];
    dit_load<S, B, VEC, NT, PT, H>(ra, base, rowstride, y);
    if (!pal) dit_load<S, B, VEC, NT, PT, H>(rb, base, rowstride, yr);
    if constexpr (PRE > 0) dit_reg_levels<S, Sh::VB, PT>(ra, pre, inverse != 0);
    dit_scatter<S, B, VEC, NT, PT>(ra, lds);
    __syncthreads();
    dit_rows_after<S, B, NT, 4, PRE>(lds, Sh::R, stages, inverse != 0, tw, pre);
    dit_store<S, B, VEC, NT, PT, H>(base, rowstride, yr, lds);
    if (!pal) {
      if constexpr (PRE > 0) dit_reg_levels<S, Sh::VB, PT>(rb, pre, inverse != 0);
      __syncthreads();  // every row of tile y's result has left LDS
      dit_scatter<S, B, VEC, NT, PT>(rb, lds);
      __syncthreads();
      dit_rows_after<S, B, NT, 4, PRE>(lds, Sh::R, stages, inverse != 0, tw, pre);
      dit_store<S, B, VEC, NT, PT, H>(base, rowstride, y, lds);
    }
    __syncthreads();
  }
}

// 16-byte accesses per thread per tile of the rectangular-tile DIT kernel:
// a thread's accesses are rows 2^BX / PT apart, so that the first log2 PT
// levels run in registers.  Measured per shape (alternating rounds, six
// levels out of place at 2^24 and 2^26): complex64 eight (three levels in
// registers); complex128 four at BX = 6 (eight held 18 more registers and
// ran 1-3% slower), two at BX = 5 (four or eight cost 1-3% at four and five
// levels).
template <int S, int BX, int BZ> constexpr int rect_pt() {
  return S == 16 ? (BX == 5 ? 2 : 4) : 8;
}

// Threads of the rectangular-tile DIT kernel, between 64 and 1024.
template <int S, int BX, int BZ> constexpr int rect_threads() {
  constexpr int c = ((1 << (BX + BZ)) * S / 16) / rect_pt<S, BX, BZ>();
  return c < 64 ? 64 : (c > 1024 ? 1024 : c);
}

// Out of place with rectangular tiles, for the fused DIT levels: the index
// is split as [x (BX bits) | y | z (BZ bits)] with BZ < BX, so rev(i) =
// [rev z | rev y | rev x].  Source tile y is 2^BX rows of 2^BZ contiguous
// elements (at a stride of 2^(m+BZ)); it lands on tile rev_m(y) of the
// destination as 2^BZ rows of 2^BX contiguous outputs (row rev(z), column
// rev(x), at a stride of 2^(m+BX)).  The levels need destination rows of at
// least 2^L outputs, which square tiles give only at 2^L rows as well; with
// BZ < BX a workgroup stages 2^(BX-BZ) times less, so more workgroups share
// a compute unit and their loads overlap each other's butterfly passes.
template <int S, int BX, int BZ, int H>
__global__ __launch_bounds__((rect_threads<S, BX, BZ>())) void k_tile_dit_rect(
    const void* src, void* dst, int m, uint64_t items_per_seg, uint64_t total_items,
    uint64_t seg_elems, int stages, int inverse, int order, int xcds) {
  typedef typename Bytes<S>::T E;
  typedef typename ComplexOf<S>::T F;
  typedef typename Bytes<16>::T V;
  constexpr int RX = 1 << BX, RZ = 1 << BZ;
  constexpr int CE = 16 / S;              // elements per 16-byte access
  constexpr int SRC_CPR = RZ / CE;        // accesses per source row
  constexpr int DST_CPR = RX / CE;        // accesses per destination row
  constexpr int CPT = RX * SRC_CPR;       // accesses per tile (either side)
  constexpr int NT = rect_threads<S, BX, BZ>();
  constexpr int PT = CPT / NT;
  constexpr int LPT = PT == 8 ? 3 : (PT == 4 ? 2 : (PT == 2 ? 1 : 0));  // log2 PT
  constexpr int PE = TileShape<S, BX, true>::PE;  // padded LDS row pitch
  constexpr int PRE = dit_reg_levels_of<CPT, SRC_CPR, NT>();
  static_assert(SRC_CPR >= 1 && CPT % NT == 0 && NT % SRC_CPR == 0 && NT % DST_CPR == 0 &&
                    (PT & (PT - 1)) == 0 && PT <= 8,
                "rectangular tile shape");
  __shared__ E lds[RZ * PE];
  __shared__ F tw[RX];
  make_twiddles<S, BX, NT>(tw);
  const uint64_t src_stride = 1ull << (m + BZ);
  const uint64_t dst_stride = 1ull << (m + BX);
  constexpr int MAXR = dit_max_radix<S, BX, false>();
  const bool pre = dit_pre_pays(stages, PRE, MAXR);  // levels 1 .. PRE in registers
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    uint64_t seg = 0, local = item;
    if (items_per_seg != total_items) {
      seg = item / items_per_seg;
      local = item - seg * items_per_seg;
    }
    const E* in = static_cast<const E*>(src) + seg * seg_elems;
    E* out = static_cast<E*>(dst) + seg * seg_elems;
    const uint32_t y = oop_tile_at(m, (uint32_t)local, order);
    // thread t reads rows x0 + i 2^BX / PT (i < PT) at column chunk zc and
    // writes destination rows r0 + i NT / DST_CPR at chunk cc: one base
    // address per side, the rest uniform steps and immediate offsets
    const uint32_t t = threadIdx.x;
    const uint32_t x0 = t / SRC_CPR, zc = t % SRC_CPR;
    const E* pin = in + (uint64_t)x0 * src_stride + (uint64_t)y * RZ + zc * CE;
    Chunk<S, 16> reg[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i)
      reg[i].v = ld_hint<H>(reinterpret_cast<const V*>(pin + (uint64_t)i * (RX / PT) * src_stride));
    if constexpr (PRE > 0) dit_reg_levels<S, 16, PT>(reg, pre, inverse != 0);
    // source (x, z) goes to LDS row rev_BZ(z), column rev_BX(x); with
    // x = x0 + i 2^(BX-LPT) the column is rev_BX(x0) + rev_LPT(i)
    const uint32_t col0 = rev_c<BX>(x0);
#pragma unroll
    for (int j = 0; j < CE; ++j) {
      E* lrow = lds + rev_c<BZ>(zc * CE + j) * PE + col0;
#pragma unroll
      for (int i = 0; i < PT; ++i) lrow[crev(i, LPT)] = reg[i].e[j];
    }
    __syncthreads();
    dit_rows_after<S, BX, NT, MAXR, PRE>(lds, RZ, stages, inverse != 0, tw, pre);
    const uint32_t yr = rev_bits(y, m);
    const uint32_t r0 = t / DST_CPR, cc = t % DST_CPR;
    const E* lsrc = lds + r0 * PE + cc * CE;
    E* pout = out + (uint64_t)r0 * dst_stride + (uint64_t)yr * RX + cc * CE;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      Chunk<S, 16> c;
#pragma unroll
      for (int j = 0; j < CE; ++j) c.e[j] = lsrc[i * (NT / DST_CPR) * PE + j];
      st_hint<H>(reinterpret_cast<V*>(pout + (uint64_t)i * (NT / DST_CPR) * dst_stride), c.v);
    }
    __syncthreads();
  }
}

template <int S, int B, bool VEC, int H>
hipError_t run_dit_h(const DitLaunch& a, hipStream_t st) {
  if (a.rs && a.t.src == a.t.dst) {
    hipLaunchKernelGGL((k_tile_dit_rs<S, B, VEC, H>), dim3(a.t.grid), dim3(rs_threads<S, B, VEC>()),
                       0, st, a.t.dst, a.t.m, a.t.items_per_seg, a.t.total_items, a.t.seg_elems,
                       a.stages, a.inverse, a.t.balanced, a.t.xcds);
    return hipGetLastError();
  }
  if (a.t.src == a.t.dst) {
    hipLaunchKernelGGL((k_tile_dit<S, B, VEC, true, H>), dim3(a.t.grid),
                       dim3(tile_threads<S, B, VEC>()), 0, st, a.t.src, a.t.dst, a.t.m,
                       a.t.items_per_seg, a.t.total_items, a.t.seg_elems, a.stages, a.inverse,
                       a.t.balanced, a.t.xcds);
  } else {
    hipLaunchKernelGGL((k_tile_dit<S, B, VEC, false, H>), dim3(a.t.grid),
                       dim3(tile_threads<S, B, VEC>()), 0, st, a.t.src, a.t.dst, a.t.m,
                       a.t.items_per_seg, a.t.total_items, a.t.seg_elems, a.stages, a.inverse,
                       a.t.balanced, a.t.xcds);
  }
  return hipGetLastError();
}

// Cache hints as for the one-item tile kernels (16-byte form only).
template <int S, int B, bool VEC>
hipError_t run_dit(const DitLaunch& a, hipStream_t st) {
  const int h = VEC ? a.t.hints : kHintPlain;
  if (h == kHintStreamLoads) return run_dit_h<S, B, VEC, kHintStreamLoads>(a, st);
  if (h == kHintStreamStores) return run_dit_h<S, B, VEC, kHintStreamStores>(a, st);
  if (h == kHintStreamWriteThrough) return run_dit_h<S, B, VEC, kHintStreamWriteThrough>(a, st);
  return run_dit_h<S, B, VEC, kHintPlain>(a, st);
}

template <int S, int BX, int BZ, int H>
hipError_t run_dit_rect_h(const DitLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((k_tile_dit_rect<S, BX, BZ, H>), dim3(a.t.grid),
                     dim3(rect_threads<S, BX, BZ>()), 0, st, a.t.src, a.t.dst, a.t.m,
                     a.t.items_per_seg, a.t.total_items, a.t.seg_elems, a.stages, a.inverse,
                     a.t.balanced, a.t.xcds);
  return hipGetLastError();
}

template <int S, int BX, int BZ>
hipError_t run_dit_rect(const DitLaunch& a, hipStream_t st) {
  switch (a.t.hints) {
    case kHintStreamLoads: return run_dit_rect_h<S, BX, BZ, kHintStreamLoads>(a, st);
    case kHintStreamStores: return run_dit_rect_h<S, BX, BZ, kHintStreamStores>(a, st);
    case kHintStreamWriteThrough: return run_dit_rect_h<S, BX, BZ, kHintStreamWriteThrough>(a, st);
    default: return run_dit_rect_h<S, BX, BZ, kHintPlain>(a, st);
  }
}

// Rectangular tiles: 2^bx source rows of 2^bz elements, bx in {5, 6},
// bz = bx - 1 or bx - 2 (16-byte aligned arrays only).
template <int S>
hipError_t dispatch_dit_rect(int bx, int bz, const DitLaunch& a, hipStream_t st) {
  if (bx == 6 && bz == 5) return run_dit_rect<S, 6, 5>(a, st);
  if (bx == 6 && bz == 4) return run_dit_rect<S, 6, 4>(a, st);
  if (bx == 5 && bz == 4) return run_dit_rect<S, 5, 4>(a, st);
  if (bx == 5 && bz == 3) return run_dit_rect<S, 5, 3>(a, st);
  return hipErrorInvalidValue;
}

template <int S, int B = 1>
hipError_t dispatch_dit(int b, bool vec, const DitLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (b == B) return vec ? run_dit<S, B, true>(a, st) : run_dit<S, B, false>(a, st);
    return dispatch_dit<S, B + 1>(b, vec, a, st);
  }
}
#endif

// Digit reversal (radix-2^D digits), in place (src == dst: pairs
// y <= drev(y)) or out of place; the tile width B and the middle width m are
// whole numbers of digits, so drev([x | y | z]) = [drev(z) | drev(y) | drev(x)].
template <int S, int B, int D, bool VEC, int H>
__global__ __launch_bounds__((tile_threads<S, B, VEC>())) void k_tile_digit(
    const void* src, void* dst, int m, uint64_t total_items, int order, int xcds) {
  static_assert(B % D == 0, "the tile width must be a whole number of digits");
  typedef typename Bytes<S>::T E;
  typedef TileShape<S, B, VEC> Sh;
  constexpr int NT = tile_threads<S, B, VEC>();
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  __shared__ E lds[2 * Sh::TILE_E];
  const bool inplace = (src == dst);
  const uint64_t rowstride = 1ull << (m + B);
  const E* in = static_cast<const E*>(src);
  E* out = static_cast<E*>(dst);
  for (uint64_t item = xcd_block(xcds); item < total_items; item += gridDim.x) {
    Chunk<S, Sh::VB> ra[PT], rb[PT];
    // out of place any order of the source tiles works (each lands on its
    // own destination tile); the order code as for the bit-reversal kernels
    const uint32_t y = inplace ? dinplace_pair_at(m, item, D) : oop_tile_at(m, (uint32_t)item, order);
    const uint32_t yr = drev_bits(y, m, D);
    const bool two = inplace && (y != yr);
    tile_load<S, B, VEC, NT, PT, H>(ra, in, rowstride, y);
    if (two) tile_load<S, B, VEC, NT, PT, H>(rb, in, rowstride, yr);
    tile_scatter<S, B, VEC, NT, PT, D>(ra, lds);
    if (two) tile_scatter<S, B, VEC, NT, PT, D>(rb, lds + Sh::TILE_E);
    __syncthreads();
    // tile y first, then its partner, as in the bit-reversal kernels
    if (two) tile_store<S, B, VEC, NT, PT, H>(out, rowstride, y, lds + Sh::TILE_E);
    tile_store<S, B, VEC, NT, PT, H>(out, rowstride, yr, lds);
    __syncthreads();
  }
}

// Digit reversal of arrays of n = 2^k <= 64: one wavefront per array.
template <int S>
__global__ __launch_bounds__(256) void k_wave_digit(const void* src, void* dst, int k, int d,
                                                    uint64_t nseg) {
  typedef typename Bytes<S>::T E;
  const int lane = (int)(threadIdx.x & 63u);
  const uint64_t n = 1ull << k;
  for (uint64_t seg = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); seg < nseg;
       seg += (uint64_t)gridDim.x * 4) {
    wave_array<S>(static_cast<const E*>(src) + seg * n, static_cast<E*>(dst) + seg * n, k, lane, d);
  }
}

// One even-odd (Stockham) split per row: evens to the first half, odds to
// the second.  A thread moves one (even, odd) pair: the loads are contiguous
// across the wavefront, and so is each of the two store streams.
template <int S>
__global__ __launch_bounds__(256) void k_evenodd(const void* src, void* dst, int k, uint64_t rows) {
  typedef typename Bytes<S>::T E;
  const uint64_t half = 1ull << (k - 1);
  const uint64_t total = half * rows;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < total; p += stride) {
    const uint64_t row = p >> (k - 1);
    const uint64_t j = p & (half - 1);
    const E* in = static_cast<const E*>(src) + (row << k) + 2 * j;
    E* out = static_cast<E*>(dst) + (row << k);
    const E a = in[0];
    const E b = in[1];
    out[j] = a;
    out[half + j] = b;
  }
}

// n = 2^k <= 64: one wavefront per array, four arrays per workgroup.
template <int S>
__global__ __launch_bounds__(256) void k_wave(const void* src, void* dst, int k, uint64_t nseg,
                                              uint64_t src_stride, uint64_t dst_stride) {
  typedef typename Bytes<S>::T E;
  const int lane = (int)(threadIdx.x & 63u);
  for (uint64_t seg = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); seg < nseg;
       seg += (uint64_t)gridDim.x * 4) {
    wave_array<S>(static_cast<const E*>(src) + seg * src_stride,
                  static_cast<E*>(dst) + seg * dst_stride, k, lane);
  }
}

// Largest a in [0, num) with scan[a] <= item, for non-decreasing scan with
// scan[0] <= item < scan[num].  Each round the 64 lanes probe 63 evenly
// spaced entries; the number that are <= item (a prefix) narrows the range
// 64-fold.  Every lane of the wavefront ends with the same answer.
__device__ __forceinline__ int64_t find_array(const int64_t* scan, int64_t num, uint64_t item) {
  const int lane = (int)(threadIdx.x & 63u);
  int64_t lo = 0, hi = num;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)(lane + 1) * step;
    const bool pred = idx < hi && (uint64_t)scan[idx] <= item;
    const int cnt = __popcll(__ballot(pred));
    lo += (int64_t)cnt * step;
    hi = (lo + step < hi) ? lo + step : hi;
  }
  return lo;
}

// Batched, in place, persistent: the prep kernel has written the exclusive
// scan of per-array work counts to ws[2..]; every workgroup walks the global
// work ids with a grid stride, finds its array and runs either the
// whole-array LDS routine (2^k < 2^(2b)) or one tile pair at width b.
template <int S, int B>
__global__ __launch_bounds__((tile_threads<S, B, true>())) void k_batched(
    void* data, const int64_t* offsets, const int32_t* log2n, int64_t num, const int64_t* ws,
    int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = tile_threads<S, B, true>();
  __shared__ E lds[2 * TileShape<S, B, true>::TILE_E];
  const int64_t* scan = ws + 2;
  const uint64_t total = (uint64_t)scan[num];
  for (uint64_t item = xcd_block(xcds); item < total; item += gridDim.x) {
    const int64_t a = find_array(scan, num, item);
    const int k = log2n[a];
    E* base = static_cast<E*>(data) + offsets[a];
    if (k < 2 * B) {
      small_array<S, NT>(base, base, k, lds);
    } else {
      const int m = k - 2 * B;
      const uint32_t y = inplace_pair_at(m, item - (uint64_t)scan[a], balanced);
      // an array after ones shorter than 16 bytes may start off the 16-byte
      // grid: it moves element by element between HBM and LDS, which keeps
      // this rare path from raising the kernel's register count (74 -> 56
      // VGPRs for complex64 at b = 6: two workgroups per CU instead of one)
      if ((reinterpret_cast<uintptr_t>(base) & 15u) == 0) {
        // streaming loads, write-through stores: 4096 complex64 arrays of
        // 2^8-2^20 elements 2.017 -> 1.947 ms (streaming stores: no gain)
        tile_pair_inplace<S, B, true, NT, kHintStreamWriteThrough, false>(base, m, y, lds);
      } else {
        tile_pair_inplace_elem<S, B, NT, 1>(base, m, y, lds);
      }
    }
    __syncthreads();
  }
}

// Batched, out of place: the same persistent walk, with one work item per
// source tile (2^m per array) or per small array; dst holds the same layout.
template <int S, int B>
__global__ __launch_bounds__((tile_threads<S, B, true>())) void k_batched_oop(
    const void* src, void* dst, const int64_t* offsets, const int32_t* log2n, int64_t num,
    const int64_t* ws, int balanced, int xcds) {
  typedef typename Bytes<S>::T E;
  constexpr int NT = tile_threads<S, B, true>();
  __shared__ E lds[2 * TileShape<S, B, true>::TILE_E];
  const int64_t* scan = ws + 2;
  const uint64_t total = (uint64_t)scan[num];
  for (uint64_t item = xcd_block(xcds); item < total; item += gridDim.x) {
    const int64_t a = find_array(scan, num, item);
    const int k = log2n[a];
    const E* in = static_cast<const E*>(src) + offsets[a];
    E* out = static_cast<E*>(dst) + offsets[a];
    if (k < 2 * B) {
      small_array<S, NT>(in, out, k, lds);
    } else {
      const int m = k - 2 * B;
      const uint32_t local = (uint32_t)(item - (uint64_t)scan[a]);
      const uint32_t y = oop_tile_at(m, local, balanced);
      if (((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0) {
        // plain accesses: write-through stores measured 1.8% slower here
        tile_outofplace<S, B, true, NT>(in, out, m, y, lds);
      } else {  // element by element, as in k_batched
        tile_outofplace_elem<S, B, NT, 1>(in, out, m, y, lds);
      }
    }
    __syncthreads();
  }
}

template <int S, int B, bool VEC, int H>
hipError_t run_inplace_h(const TileLaunch& a, hipStream_t st) {
  if (a.pipelined == 2)
    return launch_timed((k_tile_inplace_rs<S, B, VEC, H>), dim3(a.grid),
                        dim3(rs_threads<S, B, VEC>()), st, a.ev_start, a.ev_stop, a.dst, a.m,
                        a.items_per_seg, a.total_items, a.seg_elems, a.balanced, a.xcds);
  return launch_timed((k_tile_inplace<S, B, VEC, H>), dim3(a.grid),
                      dim3(tile_threads<S, B, VEC>()), st, a.ev_start, a.ev_stop, a.dst, a.m,
                      a.items_per_seg, a.total_items, a.seg_elems, a.balanced, a.xcds);
}

template <int S, int B, bool VEC>
hipError_t run_tile_inplace(const TileLaunch& a, hipStream_t st) {
  if (a.pipelined == 1)
    return launch_timed((k_tile_inplace_pipe<S, B, VEC>), dim3(a.grid),
                        dim3(tile_threads<S, B, VEC>()), st, a.ev_start, a.ev_stop, a.dst, a.m,
                        a.items_per_seg, a.total_items, a.seg_elems, a.balanced, a.xcds);
  // cache hints only on the 16-byte form; the per-element form stays plain
  const int h = VEC ? a.hints : kHintPlain;
  if (h == kHintStreamLoads) return run_inplace_h<S, B, VEC, kHintStreamLoads>(a, st);
  if (h == kHintStreamStores) return run_inplace_h<S, B, VEC, kHintStreamStores>(a, st);
  if (h == kHintStreamWriteThrough) return run_inplace_h<S, B, VEC, kHintStreamWriteThrough>(a, st);
  return run_inplace_h<S, B, VEC, kHintPlain>(a, st);
}

template <int S, int B, bool VEC, int H>
hipError_t run_outofplace_h(const TileLaunch& a, hipStream_t st) {
  return launch_timed((k_tile_outofplace<S, B, VEC, H>), dim3(a.grid),
                      dim3(tile_threads<S, B, VEC>()), st, a.ev_start, a.ev_stop, a.src, a.dst,
                      a.m, a.items_per_seg, a.total_items, a.seg_elems, a.dst_seg_elems,
                      a.balanced, a.xcds);
}

template <int S, int B, bool VEC>
hipError_t run_tile_outofplace(const TileLaunch& a, hipStream_t st) {
  if (a.pipelined == 1)
    return launch_timed((k_tile_outofplace_pipe<S, B, VEC>), dim3(a.grid),
                        dim3(tile_threads<S, B, VEC>()), st, a.ev_start, a.ev_stop, a.src, a.dst,
                        a.m, a.items_per_seg, a.total_items, a.seg_elems, a.dst_seg_elems,
                        a.balanced, a.xcds);
  const int h = VEC ? a.hints : kHintPlain;
  if (h == kHintStreamLoads) return run_outofplace_h<S, B, VEC, kHintStreamLoads>(a, st);
  if (h == kHintStreamStores) return run_outofplace_h<S, B, VEC, kHintStreamStores>(a, st);
  if (h == kHintStreamWriteThrough)
    return run_outofplace_h<S, B, VEC, kHintStreamWriteThrough>(a, st);
  return run_outofplace_h<S, B, VEC, kHintPlain>(a, st);
}

// Workgroups of a tile kernel that fit on one compute unit at once.
template <int S, int B, bool VEC>
int occupancy_of(bool inplace, bool pipelined) {
  int n = 0;
  hipError_t e;
  const int nt = tile_threads<S, B, VEC>();
  if (inplace) {
    e = pipelined ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_inplace_pipe<S, B, VEC>, nt, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_inplace<S, B, VEC, kHintPlain>, nt, 0);
  } else {
    e = pipelined ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_outofplace_pipe<S, B, VEC>, nt, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_outofplace<S, B, VEC, kHintPlain>, nt, 0);
  }
  return e == hipSuccess ? n : 0;
}

template <int S, int B>
hipError_t run_batched(const BatchedLaunch& a, hipStream_t st) {
  if (a.src != nullptr) {
    hipLaunchKernelGGL((k_batched_oop<S, B>), dim3(a.grid), dim3(tile_threads<S, B, true>()), 0, st,
                       a.src, a.data, a.offsets, a.log2n, a.num, (const int64_t*)a.ws, a.balanced,
                       a.xcds);
  } else {
    hipLaunchKernelGGL((k_batched<S, B>), dim3(a.grid), dim3(tile_threads<S, B, true>()), 0, st,
                       a.data, a.offsets, a.log2n, a.num, (const int64_t*)a.ws, a.balanced, a.xcds);
  }
  return hipGetLastError();
}

// Dispatch a runtime tile width onto the compiled instantiations.
template <int S, int B = 0>
hipError_t dispatch_tile(bool inplace, int b, bool vec, const TileLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (b == B) {
      if (inplace) return vec ? run_tile_inplace<S, B, true>(a, st) : run_tile_inplace<S, B, false>(a, st);
      return vec ? run_tile_outofplace<S, B, true>(a, st) : run_tile_outofplace<S, B, false>(a, st);
    }
    return dispatch_tile<S, B + 1>(inplace, b, vec, a, st);
  }
}

template <int S, int B, bool VEC>
hipError_t run_transpose(const TransposeLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((k_transpose_inplace<S, B, VEC>), dim3(a.grid),
                     dim3(tile_threads<S, B, VEC>()), 0, st, a.data, a.h, a.total_items, a.xcds);
  return hipGetLastError();
}

template <int S, int B = 0>
hipError_t dispatch_transpose(int b, bool vec, const TransposeLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (b == B) return vec ? run_transpose<S, B, true>(a, st) : run_transpose<S, B, false>(a, st);
    return dispatch_transpose<S, B + 1>(b, vec, a, st);
  }
}

template <int S, int D, int B = D>
hipError_t dispatch_digit(int b, bool vec, const TileLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (b == B) {
      if (vec) {
        if (a.hints == kHintStreamLoads) {
          hipLaunchKernelGGL((k_tile_digit<S, B, D, true, kHintStreamLoads>), dim3(a.grid),
                             dim3(tile_threads<S, B, true>()), 0, st, a.src, a.dst, a.m,
                             a.total_items, a.balanced, a.xcds);
        } else if (a.hints == kHintStreamStores) {
          hipLaunchKernelGGL((k_tile_digit<S, B, D, true, kHintStreamStores>), dim3(a.grid),
                             dim3(tile_threads<S, B, true>()), 0, st, a.src, a.dst, a.m,
                             a.total_items, a.balanced, a.xcds);
        } else if (a.hints == kHintStreamWriteThrough) {
          hipLaunchKernelGGL((k_tile_digit<S, B, D, true, kHintStreamWriteThrough>), dim3(a.grid),
                             dim3(tile_threads<S, B, true>()), 0, st, a.src, a.dst, a.m,
                             a.total_items, a.balanced, a.xcds);
        } else {
          hipLaunchKernelGGL((k_tile_digit<S, B, D, true, kHintPlain>), dim3(a.grid),
                             dim3(tile_threads<S, B, true>()), 0, st, a.src, a.dst, a.m,
                             a.total_items, a.balanced, a.xcds);
        }
      } else {
        hipLaunchKernelGGL((k_tile_digit<S, B, D, false, kHintPlain>), dim3(a.grid),
                           dim3(tile_threads<S, B, false>()), 0, st, a.src, a.dst, a.m,
                           a.total_items, a.balanced, a.xcds);
      }
      return hipGetLastError();
    }
    return dispatch_digit<S, D, B + D>(b, vec, a, st);
  }
}

template <int S, int B, int H>
hipError_t run_tile_copy(const TileLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((k_tile_copy<S, B, H>), dim3(a.grid), dim3(tile_threads<S, B, true>()), 0, st,
                     a.src, a.dst, a.m, a.total_items, a.balanced, a.xcds);
  return hipGetLastError();
}

template <int S, int B = 0>
hipError_t dispatch_tile_copy(int b, const TileLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (b != B) return dispatch_tile_copy<S, B + 1>(b, a, st);
    switch (a.hints) {
      case kHintStreamLoads: return run_tile_copy<S, B, kHintStreamLoads>(a, st);
      case kHintStreamStores: return run_tile_copy<S, B, kHintStreamStores>(a, st);
      case kHintStreamWriteThrough: return run_tile_copy<S, B, kHintStreamWriteThrough>(a, st);
      default: return run_tile_copy<S, B, kHintPlain>(a, st);
    }
  }
}

template <int S, int B = kMinBatchedTileBits>
hipError_t dispatch_batched(const BatchedLaunch& a, hipStream_t st) {
  if constexpr (B > max_tile_bits(S)) {
    return hipErrorInvalidValue;
  } else {
    if (a.b == B) return run_batched<S, B>(a, st);
    return dispatch_batched<S, B + 1>(a, st);
  }
}

// Workgroups of a batched kernel that fit on one compute unit at once (its
// registers can allow fewer than its LDS and thread count do).
template <int S, int B = kMinBatchedTileBits>
int batched_occupancy_for(int b, bool oop) {
  if constexpr (B > max_tile_bits(S)) {
    return 0;
  } else {
    if (b != B) return batched_occupancy_for<S, B + 1>(b, oop);
    int n = 0;
    const int nt = tile_threads<S, B, true>();
    const hipError_t e =
        oop ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched_oop<S, B>, nt, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<S, B>, nt, 0);
    return e == hipSuccess ? n : 0;
  }
}

template <int S, int B = 0>
int occupancy_for(int b, bool vec, bool inplace, bool pipelined) {
  if constexpr (B > max_tile_bits(S)) {
    return 0;
  } else {
    if (b == B) return vec ? occupancy_of<S, B, true>(inplace, pipelined) : occupancy_of<S, B, false>(inplace, pipelined);
    return occupancy_for<S, B + 1>(b, vec, inplace, pipelined);
  }
}

template <int S, int B = 0>
int threads_for(int b, bool vec) {
  if constexpr (B > max_tile_bits(S)) {
    return 0;
  } else {
    if (b == B) return vec ? tile_threads<S, B, true>() : tile_threads<S, B, false>();
    return threads_for<S, B + 1>(b, vec);
  }
}

}  // namespace

#define BITREV_CAT2(a, b) a##b
#define BITREV_CAT(a, b) BITREV_CAT2(a, b)

hipError_t BITREV_CAT(launch_tile_inplace_s, BITREV_S)(int b, bool vec, const TileLaunch& a,
                                                       hipStream_t st) {
  return dispatch_tile<BITREV_S>(true, b, vec, a, st);
}

hipError_t BITREV_CAT(launch_tile_outofplace_s, BITREV_S)(int b, bool vec, const TileLaunch& a,
                                                          hipStream_t st) {
  return dispatch_tile<BITREV_S>(false, b, vec, a, st);
}

hipError_t BITREV_CAT(launch_tile_copy_s, BITREV_S)(int b, const TileLaunch& a, hipStream_t st) {
  return dispatch_tile_copy<BITREV_S>(b, a, st);
}

hipError_t BITREV_CAT(launch_block_recursive_s, BITREV_S)(void* data, int h, uint64_t nblocks,
                                                          bool vec, uint32_t grid, hipStream_t st) {
  const size_t lds = (size_t)BITREV_S << h;
  if (vec) {
    hipLaunchKernelGGL((k_block_recursive<BITREV_S, true>), dim3(grid), dim3(512), lds, st, data, h,
                       nblocks);
  } else {
    hipLaunchKernelGGL((k_block_recursive<BITREV_S, false>), dim3(grid), dim3(512), lds, st, data,
                       h, nblocks);
  }
  return hipGetLastError();
}

hipError_t BITREV_CAT(launch_wave_s, BITREV_S)(const WaveLaunch& a, hipStream_t st) {
  hipLaunchKernelGGL((k_wave<BITREV_S>), dim3(a.grid), dim3(256), 0, st, a.src, a.dst, a.k, a.nseg,
                     a.src_stride, a.dst_stride);
  return hipGetLastError();
}

hipError_t BITREV_CAT(launch_transpose_s, BITREV_S)(int b, bool vec, const TransposeLaunch& a,
                                                    hipStream_t st) {
  return dispatch_transpose<BITREV_S>(b, vec, a, st);
}

#if BITREV_S == 8 || BITREV_S == 16
hipError_t BITREV_CAT(launch_dit_s, BITREV_S)(int b, bool vec, const DitLaunch& a, hipStream_t st) {
  if (a.rect_bz > 0) return vec ? dispatch_dit_rect<BITREV_S>(b, a.rect_bz, a, st) : hipErrorInvalidValue;
  return dispatch_dit<BITREV_S>(b, vec, a, st);
}
#endif

hipError_t BITREV_CAT(launch_digit_s, BITREV_S)(int d, int b, bool vec, const TileLaunch& a,
                                                hipStream_t st) {
  if (d == 2) return dispatch_digit<BITREV_S, 2>(b, vec, a, st);
  if (d == 3) return dispatch_digit<BITREV_S, 3>(b, vec, a, st);
  return hipErrorInvalidValue;
}

hipError_t BITREV_CAT(launch_wave_digit_s, BITREV_S)(const WaveLaunch& a, int d, hipStream_t st) {
  hipLaunchKernelGGL((k_wave_digit<BITREV_S>), dim3(a.grid), dim3(256), 0, st, a.src, a.dst, a.k, d,
                     a.nseg);
  return hipGetLastError();
}

hipError_t BITREV_CAT(launch_evenodd_s, BITREV_S)(const void* src, void* dst, int k, uint64_t rows,
                                                  uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL((k_evenodd<BITREV_S>), dim3(grid), dim3(256), 0, st, src, dst, k, rows);
  return hipGetLastError();
}

hipError_t BITREV_CAT(launch_batched_s, BITREV_S)(const BatchedLaunch& a, hipStream_t st) {
  return dispatch_batched<BITREV_S>(a, st);
}

int BITREV_CAT(tile_threads_s, BITREV_S)(int b, bool vec) { return threads_for<BITREV_S>(b, vec); }

template <int S, int B = 0>
int rs_threads_for(int b, bool vec) {
  if constexpr (B > max_tile_bits(S)) {
    return 0;
  } else {
    if (b == B) return vec ? rs_threads<S, B, true>() : rs_threads<S, B, false>();
    return rs_threads_for<S, B + 1>(b, vec);
  }
}

int BITREV_CAT(tile_rs_threads_s, BITREV_S)(int b, bool vec) { return rs_threads_for<BITREV_S>(b, vec); }

int BITREV_CAT(tile_occupancy_s, BITREV_S)(int b, bool vec, bool inplace, bool pipelined) {
  return occupancy_for<BITREV_S>(b, vec, inplace, pipelined);
}

int BITREV_CAT(batched_occupancy_s, BITREV_S)(int b, bool oop) {
  return batched_occupancy_for<BITREV_S>(b, oop);
}

int BITREV_CAT(batched_threads_s, BITREV_S)(int b) {
  return b < kMinBatchedTileBits ? 0 : threads_for<BITREV_S>(b, true);
}

}  // namespace bitrev
