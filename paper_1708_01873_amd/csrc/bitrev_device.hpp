// Device-side building blocks of libbitrev: index reversal, the work-item
// enumeration, and the per-work-item routines that the kernels in
// bitrev_kernels.hip compose.  Written for gfx950 (64-lane wavefronts).
//
// The method (arXiv:1708.01873, Introduction, bit reversal using a matrix
// buffer): split an index of k bits as i = [x | y | z] with x the high b bits,
// y the middle m = k - 2b bits and z the low b bits.  Then
// rev_k(i) = [rev_b(z) | rev_m(y) | rev_b(x)], so the 2^b x 2^b "tile" of
// elements sharing the middle bits y (rows x, each a contiguous run of 2^b
// elements z) lands as a whole on tile rev_m(y), with element (x, z) at row
// rev_b(z), column rev_b(x).  Each tile is staged through LDS so that both the
// HBM read (rows of the source tile) and the HBM write (rows of the
// destination tile) move whole contiguous rows.
//
// In place, tiles y and rev_m(y) swap (the paper's in-place variant of the
// buffered method, and the pairing by i < rev(i) of the Introduction's
// listing).  One work item owns the pair {y, rev_m(y)} with y <= rev_m(y):
// both tiles are read completely before the workgroup barrier and written
// after it, and no other work item touches either tile, so the swap is
// race-free without any global synchronisation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bitrev {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// An opaque block of N bytes held in registers.
template <int N> struct Bytes;
template <> struct Bytes<1> { typedef uint8_t T; };
template <> struct Bytes<2> { typedef uint16_t T; };
template <> struct Bytes<4> { typedef uint32_t T; };
template <> struct Bytes<8> { typedef u32x2 T; };
template <> struct Bytes<16> { typedef u32x4 T; };

// Cache hints of the tile kernels' global accesses: streaming
// (non-temporal) loads or stores mark lines the kernel touches once, so they
// do not displace other lines in L2 and the Infinity Cache.  The last form
// pairs streaming loads with write-through stores.
enum CacheHint {
  kHintPlain = 0,
  kHintStreamLoads = 1,
  kHintStreamStores = 2,
  kHintStreamWriteThrough = 3
};

template <int H, typename V> __device__ __forceinline__ V ld_hint(const V* p) {
  if constexpr (H == kHintStreamLoads || H == kHintStreamWriteThrough) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

// A store at device scope (the SC1 cache-policy bit): the line is written
// through the XCD's L2 to the memory side, where every XCD sees it, instead
// of being held dirty in that L2.  The permutation writes each line once and
// never reads it back, so nothing is lost by not keeping it; on MI355X the
// in-place tile pattern ran about 5% faster with these stores and streaming
// loads than with plain accesses.  Vector stores only; other widths store
// plainly.
//
// The compiler sees through the asm only its operands: it inserts the waits
// for the address and data registers before it, but not the wait states that
// must separate a vector store of more than 8 bytes from a later VALU write of
// its data registers (two on gfx950; without them the store can pick up the
// new value).  The asm therefore ends with its own s_nop 1 (two wait states).
template <typename V> __device__ __forceinline__ void st_through(V* p, V v) {
  if constexpr (sizeof(V) == 16) {
    asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" : : "v"(p), "v"(v) : "memory");
  } else if constexpr (sizeof(V) == 8) {
    asm volatile("global_store_dwordx2 %0, %1, off sc1\n\ts_nop 1" : : "v"(p), "v"(v) : "memory");
  } else if constexpr (sizeof(V) == 4) {
    asm volatile("global_store_dword %0, %1, off sc1\n\ts_nop 1" : : "v"(p), "v"(v) : "memory");
  } else {
    *p = v;
  }
}

template <int H, typename V> __device__ __forceinline__ void st_hint(V* p, V v) {
  if constexpr (H == kHintStreamStores) {
    __builtin_nontemporal_store(v, p);
  } else if constexpr (H == kHintStreamWriteThrough) {
    st_through(p, v);
  } else {
    *p = v;
  }
}

// VB bytes seen either as one vector or as VB/S elements of S bytes.
template <int S, int VB> union Chunk {
  typename Bytes<VB>::T v;
  typename Bytes<S>::T e[VB / S];
};

// Reverse the low j bits of v, 0 <= j <= 32 (v_bfrev_b32 and a shift).  The
// 64-bit shift makes j = 0 yield 0, the reversal of the empty bit string.
__host__ __device__ __forceinline__ uint32_t rev_bits(uint32_t v, int j) {
  return (uint32_t)(((uint64_t)__builtin_bitreverse32(v)) >> (32 - j));
}

// rev_p(v) at compile time (chunk-to-position maps of unrolled loops).
__host__ __device__ constexpr int crev(int v, int p) {
  int r = 0;
  for (int i = 0; i < p; ++i) r |= ((v >> i) & 1) << (p - 1 - i);
  return r;
}

template <int J> __host__ __device__ __forceinline__ uint32_t rev_c(uint32_t v) {
  if constexpr (J == 0) {
    return 0u;
  } else {
    return __builtin_bitreverse32(v) >> (32 - J);
  }
}

// Gather the even-position bits of w into the low half (bit 2t -> bit t).
__host__ __device__ __forceinline__ uint32_t compact_even(uint32_t w) {
  uint32_t x = w & 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}

// A bijection on width-bit values that deals the bits of w alternately to
// the low end and the high end of the field: bit 0 -> 0, bit 1 -> width-1,
// bit 2 -> 1, bit 3 -> width-2, ...  A run of consecutive w then varies both
// the low and the high bits of the result, so that consecutive work items
// touch tiles whose reversal partners are spread over HBM channels too.
__host__ __device__ __forceinline__ uint32_t spread_bits(uint32_t w, int width) {
  return compact_even(w) | rev_bits(compact_even(w >> 1), width);
}

// Number of y in [0, 2^m) with y <= rev_m(y): the r(m) swapping pairs plus
// the 2^ceil(m/2) palindromes, (2^m + 2^ceil(m/2)) / 2.
__host__ __device__ __forceinline__ uint64_t pair_count(int m) {
  return ((1ull << m) + (1ull << ((m + 1) / 2))) >> 1;
}

// The w-th y (0 <= w < pair_count(m)) with y <= rev_m(y).  Bits are decided
// from the outside in, as in the paper's branch-and-bound enumeration of
// swap pairs (Methods, unrolling): an outer pair (top, bottom) = (0, 1) makes
// y < rev(y) whatever the inner bits are; (1, 0) never qualifies; equal outer
// bits defer to the inner m - 2 bits.  Counting the three cases gives
// pair_count(m) = 2^(m-2) + 2 pair_count(m-2).  When `balanced`, the free
// inner bits are dealt by spread_bits instead of in natural order.
__host__ __device__ __forceinline__ uint32_t pair_at(int m, uint64_t w, bool balanced) {
  uint32_t y = 0;
  int lo = 0;
  int width = m;
  while (width >= 2) {
    const uint64_t q = 1ull << (width - 2);
    if (w < q) {
      uint32_t u = (uint32_t)w;
      if (balanced) u = spread_bits(u, width - 2);
      return y | (1u << lo) | (u << (lo + 1));
    }
    w -= q;
    if (w & 1) y |= (1u << lo) | (1u << (lo + width - 1));
    w >>= 1;
    lo += 1;
    width -= 2;
  }
  if (width == 1) y |= (uint32_t)(w & 1) << lo;
  return y;
}

// Number of y in [0, 2^m) with y < rev_m(y): (2^m - 2^ceil(m/2)) / 2 (the
// paper's swap count r, Methods, unrolling).  pair_at lists exactly these
// for w < swap_pair_count(m), before any palindrome.
__host__ __device__ __forceinline__ uint64_t swap_pair_count(int m) {
  return ((1ull << m) - (1ull << ((m + 1) / 2))) >> 1;
}

// The t-th palindrome y = rev_m(y), 0 <= t < 2^ceil(m/2).
__host__ __device__ __forceinline__ uint32_t palindrome_at(int m, uint32_t t) {
  const int h = m >> 1;
  if (m & 1) return ((t >> 1) << (h + 1)) | ((t & 1u) << h) | rev_bits(t >> 1, h);
  return (t << h) | rev_bits(t, h);
}

// Grouped order of the in-place tile pairs (1 <= j, 2j <= m).  The m tile
// bits are split as y = [t | c | s] (t and s of j bits), so that
// rev_m(y) = [rev_j(s) | rev(c) | rev_j(t)].  A middle c < rev(c) owns the
// 4^j pairs {[t|c|s], rev_m([t|c|s])} for all (t, s); a palindromic middle
// owns the pairs of the 2j-bit values [t|s] under their own reversal.
// Consecutive work items then cover 2^j neighbouring tiles on both sides of
// the swap, where pair_at's outside-in order leaves a hole after every tile.
// Returns one tile of the w-th pair (0 <= w < pair_count(m)); the other is
// its reversal.
__host__ __device__ __forceinline__ uint32_t group_pair_at(int m, int j, uint64_t w,
                                                           bool balanced) {
  const int mc = m - 2 * j;
  const uint64_t per = 1ull << (2 * j);
  const uint64_t r = swap_pair_count(mc);
  uint32_t c, z;
  if (w < r * per) {
    c = pair_at(mc, w >> (2 * j), balanced);
    z = (uint32_t)(w & (per - 1));
  } else {
    const uint64_t w2 = w - r * per;
    const uint64_t pp = pair_count(2 * j);
    const uint64_t g = w2 / pp;
    c = palindrome_at(mc, (uint32_t)g);
    z = pair_at(2 * j, w2 - g * pp, false);
  }
  const uint32_t t = z >> j, sb = z & ((1u << j) - 1u);
  return (t << (mc + j)) | (c << j) | sb;
}

// The in-place kernels' order code: bit 0 balanced, bits 1.. the group
// width j (0: pair_at's own order), at most m / 2 for an m-bit middle.
__host__ __device__ __forceinline__ uint32_t inplace_pair_at(int m, uint64_t w, int order_code) {
  const int j = (order_code >> 1) < (m >> 1) ? (order_code >> 1) : (m >> 1);
  const bool bal = (order_code & 1) != 0;
  return j ? group_pair_at(m, j, w, bal) : pair_at(m, w, bal);
}

// The w-th source tile of the out-of-place kernels for an order code (see
// inplace_pair_at).  Grouped: y = [t | c | s] with (s, t) the low 2j bits of
// w, s fastest, and the middle c dealt by spread_bits from the rest, so that
// each run of 4^j items covers 2^j neighbouring tiles on both sides.
__host__ __device__ __forceinline__ uint32_t oop_tile_at(int m, uint32_t w, int order_code) {
  const int j = (order_code >> 1) < (m >> 1) ? (order_code >> 1) : (m >> 1);
  if (j == 0) return (order_code & 1) ? spread_bits(w, m) : w;
  const int mc = m - 2 * j;
  const uint32_t s = w & ((1u << j) - 1u);
  const uint32_t t = (w >> j) & ((1u << j) - 1u);
  const uint32_t c = spread_bits(w >> (2 * j), mc);
  return (t << (mc + j)) | (c << j) | s;
}

// ---------------------------------------------------------------------------
// Digit reversal for radix-2^D FFTs: the order of the D-bit digits of an
// index is reversed, each digit keeping its own bits.  D = 1 is rev_bits.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t drev_bits(uint32_t v, int j, int d) {
  uint32_t r = 0;
  const uint32_t mask = (1u << d) - 1u;
  for (int t = 0; t < j; t += d) r = (r << d) | ((v >> t) & mask);
  return r;
}

template <int J, int D> __host__ __device__ __forceinline__ uint32_t drev_c(uint32_t v) {
  if constexpr (D == 1) {
    return rev_c<J>(v);
  } else {
    uint32_t r = 0;
#pragma unroll
    for (int t = 0; t < J; t += D) r = (r << D) | ((v >> t) & ((1u << D) - 1u));
    return r;
  }
}

// y in [0, 2^m) with y <= drev(y): (q^(m/d) + q^ceil(m/(2d))) / 2, q = 2^d.
__host__ __device__ __forceinline__ uint64_t dpair_count(int m, int d) {
  const int digits = m / d;
  return ((1ull << m) + (1ull << (d * ((digits + 1) / 2)))) >> 1;
}

// The w-th y with y <= drev(y), digits decided from the outside in: an outer
// digit pair (top T, bottom U) with T < U makes y < drev(y) for any inner
// digits, T > U never does, T = U defers to the inner digits -- the
// branch-and-bound rule of the paper's unrolled method (Methods, unrolling)
// with digits in place of bits.
__host__ __device__ __forceinline__ uint32_t dpair_at(int m, uint64_t w, int d) {
  const uint32_t q = 1u << d;
  uint32_t y = 0;
  int lo = 0;
  int width = m;
  while (width >= 2 * d) {
    const int inner = width - 2 * d;
    const uint64_t q2 = ((uint64_t)(q * (q - 1) / 2)) << inner;
    if (w < q2) {
      const uint32_t p = (uint32_t)(w >> inner);
      const uint32_t u = (uint32_t)(w & ((1ull << inner) - 1));
      uint32_t hi_d = 1;  // pairs (lo_d < hi_d) number hi_d (hi_d - 1) / 2 before hi_d
      while ((hi_d + 1) * hi_d / 2 <= p) ++hi_d;
      const uint32_t lo_d = p - hi_d * (hi_d - 1) / 2;
      return y | (hi_d << lo) | (lo_d << (lo + width - d)) | (u << (lo + d));
    }
    w -= q2;
    const uint32_t e = (uint32_t)(w % q);
    w /= q;
    y |= (e << lo) | (e << (lo + width - d));
    lo += d;
    width -= 2 * d;
  }
  if (width == d) y |= (uint32_t)w << lo;
  return y;
}

// Number of y with y < drev(y): (2^m - q^ceil(m/(2d))) / 2.  As for
// pair_at, dpair_at lists exactly these first (w < dswap_pair_count).
__host__ __device__ __forceinline__ uint64_t dswap_pair_count(int m, int d) {
  const int digits = m / d;
  return ((1ull << m) - (1ull << (d * ((digits + 1) / 2)))) >> 1;
}

// The t-th y with y = drev(y), 0 <= t < q^ceil(m/(2d)): the high digits
// (and, for an odd digit count, the middle digit) come from t, the low
// digits are the high ones in reverse order.
__host__ __device__ __forceinline__ uint32_t dpalindrome_at(int m, uint32_t t, int d) {
  const int digits = m / d;
  const int h = digits / 2;
  const uint32_t top = (digits & 1) ? t >> d : t;
  const uint32_t mid = (digits & 1) ? t & ((1u << d) - 1u) : 0u;
  return (top << (m - h * d)) | (mid << (h * d)) | drev_bits(top, h * d, d);
}

// The grouped order of group_pair_at with digits: y = [t | c | s], t and s
// of j digits, drev(y) = [drev(s) | drev(c) | drev(t)]; a middle
// c < drev(c) owns all (t, s), a digit palindrome c the pairs of the
// 2j-digit [t|s] under its own digit reversal.  2jd <= m.
__host__ __device__ __forceinline__ uint32_t dgroup_pair_at(int m, uint64_t w, int d, int j) {
  const int gb = j * d;
  const int mc = m - 2 * gb;
  const uint64_t per = 1ull << (2 * gb);
  const uint64_t r = dswap_pair_count(mc, d);
  uint32_t c, z;
  if (w < r * per) {
    c = dpair_at(mc, w >> (2 * gb), d);
    z = (uint32_t)(w & (per - 1));
  } else {
    const uint64_t w2 = w - r * per;
    const uint64_t pp = dpair_count(2 * gb, d);
    const uint64_t g = w2 / pp;
    c = dpalindrome_at(mc, (uint32_t)g, d);
    z = dpair_at(2 * gb, w2 - g * pp, d);
  }
  const uint32_t t = z >> gb, sb = z & ((1u << gb) - 1u);
  return (t << (mc + gb)) | (c << gb) | sb;
}

// The digit kernels' in-place order: grouped with about 3 bits per side
// (ceil(3 / d) digits), fewer where the middle is short, dpair_at's own
// order when not even one digit per side fits.
__host__ __device__ __forceinline__ uint32_t dinplace_pair_at(int m, uint64_t w, int d) {
  int j = (3 + d - 1) / d;
  if (2 * j * d > m) j = m / (2 * d);
  return j ? dgroup_pair_at(m, w, d, j) : dpair_at(m, w, d);
}

// LDS padding per tile row, in elements: one element (at least 4 bytes)
// staggers consecutive rows across banks for the column-wise scatter.
__host__ __device__ constexpr int lds_pad_elems(int s) { return s >= 4 ? 1 : 4 / s; }

// LDS bytes of `tiles` staged tiles of width b for s-byte elements.
__host__ __device__ constexpr size_t tile_lds_bytes_for(int s, int b, int tiles) {
  return (size_t)tiles * ((size_t)1 << b) * (((size_t)1 << b) + (size_t)lds_pad_elems(s)) * (size_t)s;
}

// The tile geometry for element size S, tile width B and access mode.
// VEC: global memory moves 16-byte vectors (or whole rows, if shorter);
// otherwise one element per access (used when a base pointer is not
// 16-byte aligned).
template <int S, int B, bool VEC> struct TileShape {
  static constexpr int R = 1 << B;                  // rows per tile = elements per row
  static constexpr int ROWB = R * S;                // bytes per row
  static constexpr int VB = VEC ? (ROWB < 16 ? ROWB : 16) : S;  // bytes per access
  static constexpr int CE = VB / S;                 // elements per access
  static constexpr int CPR = R / CE;                // accesses per row
  static constexpr int CPT = R * CPR;               // accesses per tile
  static constexpr int PADE = lds_pad_elems(S);
  static constexpr int PE = R + PADE;               // LDS row pitch, elements
  static constexpr int TILE_E = R * PE;             // LDS elements per tile
};

// Threads per workgroup for a tile kernel: two accesses per thread per tile,
// between one wavefront and 1024 threads.
template <int S, int B, bool VEC> constexpr int tile_threads() {
  constexpr int c = TileShape<S, B, VEC>::CPT / 2;
  return c < 64 ? 64 : (c > 1024 ? 1024 : c);
}

// Threads per workgroup of the register-staged in-place kernel: four
// accesses per thread per tile (half the plain kernel's threads), so that
// twice as many workgroups, each holding its tile pair in registers, fit on
// a compute unit.
template <int S, int B, bool VEC> constexpr int rs_threads() {
  constexpr int c = TileShape<S, B, VEC>::CPT / 4;
  return c < 64 ? 64 : (c > 512 ? 512 : c);
}

// Logical block index: the hardware deals workgroups to the XCDs round
// robin, so block i runs on XCD i % xcds.  Renumber so that each XCD owns a
// contiguous range of work items; neighbouring work items then share its L2
// and spread over its channels.  grid must be a multiple of xcds.
__device__ __forceinline__ uint32_t xcd_block(int xcds) {
  const uint32_t g = gridDim.x / (uint32_t)xcds;
  return (blockIdx.x % (uint32_t)xcds) * g + blockIdx.x / (uint32_t)xcds;
}

// ---------------------------------------------------------------------------
// Tile routines.  All threads of the workgroup call them together; `lds`
// holds room for two tiles.
// ---------------------------------------------------------------------------

// Load one tile (middle bits y) of the array at `base` into registers.
template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_load(Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                          const typename Bytes<S>::T* __restrict__ base,
                                          uint64_t rowstride, uint32_t y) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<Sh::VB>::T V;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    if (Sh::CPT % NT == 0 || q < Sh::CPT) {
      const int x = q / Sh::CPR;
      const int zc = q % Sh::CPR;
      const uint64_t off = (uint64_t)x * rowstride + (uint64_t)y * Sh::R + (uint64_t)(zc * Sh::CE);
      reg[i].v = ld_hint<H>(reinterpret_cast<const V*>(base + off));
    }
  }
}

// Scatter registers into LDS in destination order: source (x, z) goes to
// LDS row rev_b(z), column rev_b(x).  MAP selects the index map: 1 the bit
// reversal, D > 1 the reversal of D-bit digits, 0 none (the plain square
// transpose: row z, column x).
template <int S, int B, bool VEC, int NT, int PT, int MAP = 1>
__device__ __forceinline__ void tile_scatter(const Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                             typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    if (Sh::CPT % NT == 0 || q < Sh::CPT) {
      const int x = q / Sh::CPR;
      const int zc = q % Sh::CPR;
      const uint32_t col = MAP ? drev_c<B, (MAP ? MAP : 1)>((uint32_t)x) : (uint32_t)x;
#pragma unroll
      for (int j = 0; j < Sh::CE; ++j) {
        const uint32_t z = (uint32_t)(zc * Sh::CE + j);
        const uint32_t row = MAP ? drev_c<B, (MAP ? MAP : 1)>(z) : z;
        lds[row * Sh::PE + col] = reg[i].e[j];
      }
    }
  }
}

// Write the staged tile (destination order in LDS) to tile y of `base`.
template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_store(typename Bytes<S>::T* __restrict__ base,
                                           uint64_t rowstride, uint32_t y,
                                           const typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<Sh::VB>::T V;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    if (Sh::CPT % NT == 0 || q < Sh::CPT) {
      const int r = q / Sh::CPR;
      const int cc = q % Sh::CPR;
      Chunk<S, Sh::VB> c;
#pragma unroll
      for (int j = 0; j < Sh::CE; ++j) c.e[j] = lds[r * Sh::PE + cc * Sh::CE + j];
      const uint64_t off = (uint64_t)r * rowstride + (uint64_t)y * Sh::R + (uint64_t)(cc * Sh::CE);
      st_hint<H>(reinterpret_cast<V*>(base + off), c.v);
    }
  }
}

// tile_load, tile_scatter (bit reversal) and tile_store for thread counts
// that are a multiple of the accesses per row: thread t's chunk i is then
// row x0 + i NT / CPR (x0 = t / CPR, the top log2 PT bits of the row index
// are i) at chunk t % CPR, so every address is one per-thread base plus
// uniform steps and immediate offsets.  (From the general forms the
// compiler keeps PT 64-bit row offsets live across the item loop.)
template <int S, int B, bool VEC, int NT, int PT>
constexpr bool tile_rows_strided() {
  typedef TileShape<S, B, VEC> Sh;
  return Sh::CPT == NT * PT && NT % Sh::CPR == 0 && (PT & (PT - 1)) == 0;
}

template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_load_rows(Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                               const typename Bytes<S>::T* __restrict__ base,
                                               uint64_t rowstride, uint32_t y) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<Sh::VB>::T V;
  static_assert(tile_rows_strided<S, B, VEC, NT, PT>(), "strided row assignment");
  const uint32_t t = threadIdx.x;
  const typename Bytes<S>::T* p = base + (uint64_t)(t / Sh::CPR) * rowstride +
                                  (uint64_t)y * Sh::R + (t % Sh::CPR) * Sh::CE;
#pragma unroll
  for (int i = 0; i < PT; ++i)
    reg[i].v = ld_hint<H>(reinterpret_cast<const V*>(p + (uint64_t)i * (NT / Sh::CPR) * rowstride));
}

template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void tile_scatter_rows(
    const Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT], typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  static_assert(tile_rows_strided<S, B, VEC, NT, PT>(), "strided row assignment");
  constexpr int LPT = PT >= 8 ? 3 : (PT == 4 ? 2 : (PT == 2 ? 1 : 0));
  static_assert((1 << LPT) == PT, "two to eight chunks per thread");
  const uint32_t t = threadIdx.x;
  // source (x, z) -> LDS row rev_B(z), column rev_B(x); x = x0 + i 2^(B-LPT)
  // has column rev_B(x0) + rev_LPT(i)
  const uint32_t col0 = rev_c<B>(t / Sh::CPR);
#pragma unroll
  for (int j = 0; j < Sh::CE; ++j) {
    typename Bytes<S>::T* lrow = lds + rev_c<B>((t % Sh::CPR) * Sh::CE + j) * Sh::PE + col0;
#pragma unroll
    for (int i = 0; i < PT; ++i) lrow[crev(i, LPT)] = reg[i].e[j];
  }
}

template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_store_rows(typename Bytes<S>::T* __restrict__ base,
                                                uint64_t rowstride, uint32_t y,
                                                const typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<Sh::VB>::T V;
  static_assert(tile_rows_strided<S, B, VEC, NT, PT>(), "strided row assignment");
  const uint32_t t = threadIdx.x;
  const uint32_t r0 = t / Sh::CPR, cc = t % Sh::CPR;
  const typename Bytes<S>::T* l = lds + r0 * Sh::PE + cc * Sh::CE;
  typename Bytes<S>::T* p = base + (uint64_t)r0 * rowstride + (uint64_t)y * Sh::R + cc * Sh::CE;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    Chunk<S, Sh::VB> c;
#pragma unroll
    for (int j = 0; j < Sh::CE; ++j) c.e[j] = l[i * (NT / Sh::CPR) * Sh::PE + j];
    st_hint<H>(reinterpret_cast<V*>(p + (uint64_t)i * (NT / Sh::CPR) * rowstride), c.v);
  }
}

// LDS -> registers in the order tile_store writes: chunk i of this thread
// is LDS row r, chunk cc (destination row r of the tile).
template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void tile_gather(Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                            const typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    if (Sh::CPT % NT == 0 || q < Sh::CPT) {
      const int r = q / Sh::CPR;
      const int cc = q % Sh::CPR;
#pragma unroll
      for (int j = 0; j < Sh::CE; ++j) reg[i].e[j] = lds[r * Sh::PE + cc * Sh::CE + j];
    }
  }
}

// ---------------------------------------------------------------------------
// Swizzled LDS stage of the bit-reversal tile kernels for 8-byte elements
// moved as 16-byte vectors.  An LDS row is 2^L 16-byte slots (L = b - 1) with
// no padding, and logical slot c of row r is stored at slot c ^ swz_key(r).
//
// A thread holds chunk q and chunk q + CPT/2, i.e. source rows x and
// x + R/2 at the same chunk index zc, whose destination columns rev_b(x) and
// rev_b(x) + 1 are adjacent: each scatter write is one 16-byte slot, half the
// LDS writes of the element-wise scatter.  The lanes of a wavefront hold
// consecutive zc of one source row, bound for destination rows
// r = rev_b(2 zc + j); the low L bits of such an r are rev_L(zc), and the key
// spreads their slots over distinct banks (with the bit-reversal key,
// swz_key(r) = zc).  The row-order reads (2^L lanes per row, XORed by one
// constant) are distinct slots too, and the key is chosen so that the rows
// one read instruction gathers do not make it take a second pass (see
// swz_key).  The padded layout's element-wise scatter lost half its LDS
// cycles to bank conflicts.  The tiles sit at the same offsets as in the
// padded layout (a tile's pad is left unused).  16-byte elements keep the
// padded layout: the same swizzle measured up to 2% slower for them.
// ---------------------------------------------------------------------------
template <int S, int B, bool VEC, int NT> constexpr bool lds_swizzled() {
  typedef TileShape<S, B, VEC> Sh;
  if (S != 8 || !VEC || Sh::VB != 16) return false;
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  return Sh::CPT % NT == 0 && PT % 2 == 0;
}

// The XOR key of LDS row r in the swizzled layout (L = b - 1 slot bits): the
// physical slot of logical slot c is c ^ key(r).  Writes of 16 bytes are
// served 8 lanes at a time and need 8 distinct slots modulo 8; reads of 16
// bytes are served a quarter of a wavefront at a time, and on gfx950 they
// ran conflict-free only when the four 16-lane groups of one read agree in
// the key's bits 2-3 (a probe of XOR patterns on 256-byte rows: keys that
// differ in bits 0-1 between the groups cost nothing, in bit 2 or 3 a
// second pass).  At b = 5 a wavefront gathers four consecutive rows, so the
// key keeps bits 2-3 of r and folds bit 3 into bit 0: r ^ (r >> 3); the
// scatter's eight lanes still land on eight distinct slots modulo 8.  The
// bit reversal (b = 4, 6) was conflict-free there and stays.
template <int L> __device__ __forceinline__ uint32_t swz_key(uint32_t r) {
  const uint32_t lo = r & ((1u << L) - 1u);
  if constexpr (L == 4) {
    return lo ^ (lo >> 3);
  } else {
    return rev_c<L>(lo);
  }
}

template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void tile_scatter_swz(const Chunk<S, 16> (&reg)[PT],
                                                 typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<16>::T V;
  constexpr int L = B - 1;
  constexpr int HALF = PT / 2;
  V* l = reinterpret_cast<V*>(lds);
#pragma unroll
  for (int i = 0; i < HALF; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    const uint32_t x = (uint32_t)(q / Sh::CPR);  // < R/2; chunk i + HALF is row x + R/2
    const uint32_t zc = (uint32_t)(q % Sh::CPR);
    // both destination rows rev_b(2 zc) and rev_b(2 zc + 1) are rev_L(zc)
    // modulo 2^L, so one key serves the two stores
    const uint32_t slot = (rev_c<B>(x) >> 1) ^ swz_key<L>(rev_c<L>(zc));
    // element j of both chunks, as whole-vector shuffles (a union copy here
    // sends the register arrays to scratch memory)
    const V a = reg[i].v, b = reg[i + HALF].v;
    l[(rev_c<B>(2u * zc) << L) + slot] = __builtin_shufflevector(a, b, 0, 1, 4, 5);
    l[(rev_c<B>(2u * zc + 1u) << L) + slot] = __builtin_shufflevector(a, b, 2, 3, 6, 7);
  }
}

// Swizzled counterpart of tile_store.
template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_store_swz(typename Bytes<S>::T* __restrict__ base,
                                               uint64_t rowstride, uint32_t y,
                                               const typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<16>::T V;
  constexpr int L = B - 1;
  const V* l = reinterpret_cast<const V*>(lds);
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    const uint32_t r = (uint32_t)(q / Sh::CPR);
    const uint32_t cc = (uint32_t)(q % Sh::CPR);
    const V v = l[(r << L) + (cc ^ swz_key<L>(r))];
    const uint64_t off = (uint64_t)r * rowstride + (uint64_t)y * Sh::R + (uint64_t)(cc * Sh::CE);
    st_hint<H>(reinterpret_cast<V*>(base + off), v);
  }
}

// Swizzled counterpart of tile_gather.
template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void tile_gather_swz(Chunk<S, 16> (&reg)[PT],
                                                const typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<16>::T V;
  constexpr int L = B - 1;
  const V* l = reinterpret_cast<const V*>(lds);
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    const uint32_t r = (uint32_t)(q / Sh::CPR);
    const uint32_t cc = (uint32_t)(q % Sh::CPR);
    reg[i].v = l[(r << L) + (cc ^ swz_key<L>(r))];
  }
}

// The bit-reversal LDS stage: swizzled where lds_swizzled holds, padded
// otherwise.  Scatter in destination order, then store or gather by rows.
template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void rev_scatter(const Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                            typename Bytes<S>::T* lds) {
  if constexpr (lds_swizzled<S, B, VEC, NT>()) {
    tile_scatter_swz<S, B, VEC, NT, PT>(reg, lds);
  } else {
    tile_scatter<S, B, VEC, NT, PT>(reg, lds);
  }
}

template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void rev_store(typename Bytes<S>::T* __restrict__ base,
                                          uint64_t rowstride, uint32_t y,
                                          const typename Bytes<S>::T* lds) {
  if constexpr (lds_swizzled<S, B, VEC, NT>()) {
    tile_store_swz<S, B, VEC, NT, PT, H>(base, rowstride, y, lds);
  } else {
    tile_store<S, B, VEC, NT, PT, H>(base, rowstride, y, lds);
  }
}

template <int S, int B, bool VEC, int NT, int PT>
__device__ __forceinline__ void rev_gather(Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                           const typename Bytes<S>::T* lds) {
  if constexpr (lds_swizzled<S, B, VEC, NT>()) {
    tile_gather_swz<S, B, VEC, NT, PT>(reg, lds);
  } else {
    tile_gather<S, B, VEC, NT, PT>(reg, lds);
  }
}

// Registers (as tile_gather left them) -> the rows of tile y in HBM.
template <int S, int B, bool VEC, int NT, int PT, int H = kHintPlain>
__device__ __forceinline__ void tile_put(const Chunk<S, TileShape<S, B, VEC>::VB> (&reg)[PT],
                                         typename Bytes<S>::T* __restrict__ base,
                                         uint64_t rowstride, uint32_t y) {
  typedef TileShape<S, B, VEC> Sh;
  typedef typename Bytes<Sh::VB>::T V;
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int q = (int)threadIdx.x + i * NT;
    if (Sh::CPT % NT == 0 || q < Sh::CPT) {
      const int r = q / Sh::CPR;
      const int cc = q % Sh::CPR;
      const uint64_t off = (uint64_t)r * rowstride + (uint64_t)y * Sh::R + (uint64_t)(cc * Sh::CE);
      st_hint<H>(reinterpret_cast<V*>(base + off), reg[i].v);
    }
  }
}

// In place through one LDS tile: both tiles of the pair are read into
// registers, then each in turn is scattered into LDS and gathered back in
// destination order, and both are written.  Half the LDS of
// tile_pair_inplace and twice the registers per thread, so that twice as
// many pairs are in flight per compute unit.  Ends with the LDS free for the
// next item only after the caller's barrier.
template <int S, int B, bool VEC, int NT, int H = kHintPlain>
__device__ __forceinline__ void tile_pair_inplace_rs(typename Bytes<S>::T* __restrict__ base,
                                                     int m, uint32_t y,
                                                     typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  const uint64_t rowstride = 1ull << (m + B);
  const uint32_t yr = rev_bits(y, m);
  const bool pal = (yr == y);
  Chunk<S, Sh::VB> ra[PT], rb[PT];
  tile_load<S, B, VEC, NT, PT, H>(ra, base, rowstride, y);
  if (!pal) tile_load<S, B, VEC, NT, PT, H>(rb, base, rowstride, yr);
  rev_scatter<S, B, VEC, NT, PT>(ra, lds);
  __syncthreads();
  rev_gather<S, B, VEC, NT, PT>(ra, lds);  // tile y, transposed: its rows go to yr
  if (!pal) {
    __syncthreads();
    rev_scatter<S, B, VEC, NT, PT>(rb, lds);
    __syncthreads();
    rev_gather<S, B, VEC, NT, PT>(rb, lds);
    tile_put<S, B, VEC, NT, PT, H>(rb, base, rowstride, y);
  }
  tile_put<S, B, VEC, NT, PT, H>(ra, base, rowstride, yr);
}

// Element-wise tiles with more accesses per thread than registers can hold
// (an array that is not 16-byte aligned, at a wide tile): elements go from
// HBM straight into LDS in destination order and from LDS straight back, one
// at a time, with no register staging.  In place, both tiles sit in LDS
// before the barrier and are written after it.
template <int S, int B, bool VEC, int NT> constexpr bool tile_elementwise() {
  return !VEC && (TileShape<S, B, VEC>::CPT + NT - 1) / NT > 8;
}

// U is the unroll depth of the element loops: 4 where this routine is the
// kernel's main path, 1 where it is a rare fallback that must not raise the
// kernel's register count (the batched kernels).
template <int S, int B, int NT, int U = 4>
__device__ __forceinline__ void tile_pair_inplace_elem(typename Bytes<S>::T* __restrict__ base,
                                                       int m, uint32_t y,
                                                       typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, false> Sh;
  const uint64_t rowstride = 1ull << (m + B);
  const uint32_t yr = rev_bits(y, m);
  const bool pal = (yr == y);
#pragma unroll U
  for (int q = (int)threadIdx.x; q < Sh::CPT; q += NT) {
    const uint32_t x = (uint32_t)q >> B, z = (uint32_t)q & (Sh::R - 1);
    const uint32_t d = rev_c<B>(z) * Sh::PE + rev_c<B>(x);
    const uint64_t off = (uint64_t)x * rowstride + z;
    lds[d] = base[off + (uint64_t)y * Sh::R];
    if (!pal) lds[Sh::TILE_E + d] = base[off + (uint64_t)yr * Sh::R];
  }
  __syncthreads();
#pragma unroll U
  for (int q = (int)threadIdx.x; q < Sh::CPT; q += NT) {
    const uint32_t r = (uint32_t)q >> B, c = (uint32_t)q & (Sh::R - 1);
    const uint64_t off = (uint64_t)r * rowstride + c;
    if (!pal) base[off + (uint64_t)y * Sh::R] = lds[Sh::TILE_E + r * Sh::PE + c];
    base[off + (uint64_t)yr * Sh::R] = lds[r * Sh::PE + c];
  }
}

template <int S, int B, int NT, int U = 4>
__device__ __forceinline__ void tile_outofplace_elem(const typename Bytes<S>::T* __restrict__ src,
                                                     typename Bytes<S>::T* __restrict__ dst,
                                                     int m, uint32_t y,
                                                     typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, false> Sh;
  const uint64_t rowstride = 1ull << (m + B);
  const uint32_t yr = rev_bits(y, m);
#pragma unroll U
  for (int q = (int)threadIdx.x; q < Sh::CPT; q += NT) {
    const uint32_t x = (uint32_t)q >> B, z = (uint32_t)q & (Sh::R - 1);
    lds[rev_c<B>(z) * Sh::PE + rev_c<B>(x)] = src[(uint64_t)x * rowstride + (uint64_t)y * Sh::R + z];
  }
  __syncthreads();
#pragma unroll U
  for (int q = (int)threadIdx.x; q < Sh::CPT; q += NT) {
    const uint32_t r = (uint32_t)q >> B, c = (uint32_t)q & (Sh::R - 1);
    dst[(uint64_t)r * rowstride + (uint64_t)yr * Sh::R + c] = lds[r * Sh::PE + c];
  }
}

// In place: swap tiles y and yr = rev_m(y) of the array at `base` (one tile
// when y is a palindrome).  Ends with the LDS free for the next item only
// after the caller's barrier.  SERIAL: the partner's loads are issued only
// once tile y has arrived and is scattered, rather than together with tile
// y's.  Alternating rounds, kernel time, caches evicted: at b = 5 +1.6%
// (complex64 2^24) and +0.6% (complex128 2^28); float32 at b = 6 +0.3% to
// +2.2% (2^24 to 2^30); complex64 at b = 6 -1.3% (2^26) to +0.6% (2^29),
// so it keeps the joint loads.
template <int S, int B, bool VEC, int NT, int H = kHintPlain, bool SERIAL = (B <= 5 || S == 4)>
__device__ __forceinline__ void tile_pair_inplace(typename Bytes<S>::T* __restrict__ base, int m,
                                                  uint32_t y, typename Bytes<S>::T* lds) {
  if constexpr (tile_elementwise<S, B, VEC, NT>()) {
    tile_pair_inplace_elem<S, B, NT>(base, m, y, lds);
    return;
  }
  typedef TileShape<S, B, VEC> Sh;
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  const uint64_t rowstride = 1ull << (m + B);
  const uint32_t yr = rev_bits(y, m);
  const bool pal = (yr == y);
  Chunk<S, Sh::VB> ra[PT], rb[PT];
  tile_load<S, B, VEC, NT, PT, H>(ra, base, rowstride, y);
  if constexpr (SERIAL) {
    rev_scatter<S, B, VEC, NT, PT>(ra, lds);
    if (!pal) {
      tile_load<S, B, VEC, NT, PT, H>(rb, base, rowstride, yr);
      rev_scatter<S, B, VEC, NT, PT>(rb, lds + Sh::TILE_E);
    }
  } else {
    if (!pal) tile_load<S, B, VEC, NT, PT, H>(rb, base, rowstride, yr);
    rev_scatter<S, B, VEC, NT, PT>(ra, lds);
    if (!pal) rev_scatter<S, B, VEC, NT, PT>(rb, lds + Sh::TILE_E);
  }
  __syncthreads();
  // tile y first, then its partner: measured a few percent faster than the
  // other order for arrays that fit the Infinity Cache
  if (!pal) rev_store<S, B, VEC, NT, PT, H>(base, rowstride, y, lds + Sh::TILE_E);
  rev_store<S, B, VEC, NT, PT, H>(base, rowstride, yr, lds);
}

// Out of place: tile y of `src` to tile rev_m(y) of `dst`.
template <int S, int B, bool VEC, int NT, int H = kHintPlain>
__device__ __forceinline__ void tile_outofplace(const typename Bytes<S>::T* __restrict__ src,
                                                typename Bytes<S>::T* __restrict__ dst, int m,
                                                uint32_t y, typename Bytes<S>::T* lds) {
  if constexpr (tile_elementwise<S, B, VEC, NT>()) {
    tile_outofplace_elem<S, B, NT>(src, dst, m, y, lds);
    return;
  }
  typedef TileShape<S, B, VEC> Sh;
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  const uint64_t rowstride = 1ull << (m + B);
  Chunk<S, Sh::VB> ra[PT];
  tile_load<S, B, VEC, NT, PT, H>(ra, src, rowstride, y);
  rev_scatter<S, B, VEC, NT, PT>(ra, lds);
  __syncthreads();
  rev_store<S, B, VEC, NT, PT, H>(dst, rowstride, rev_bits(y, m), lds);
}

// ---------------------------------------------------------------------------
// Fused first FFT levels.  After the reversal, a radix-2 decimation-in-time
// FFT works on contiguous blocks (Introduction: every even-odd split done up
// front is the bit-reversed permutation).  Each LDS row of a staged tile is a
// contiguous run of 2^b outputs starting at a multiple of 2^b, so the first
// L <= b levels run on the staged rows before they are written: the blocks
// of 2^L outputs leave as length-2^L DFTs, at no extra HBM traffic.
// ---------------------------------------------------------------------------
template <int S> struct ComplexOf;
template <> struct ComplexOf<8> { typedef float T; };
template <> struct ComplexOf<16> { typedef double T; };

// One complex element as a single naturally aligned store.
template <typename F> struct alignas(2 * sizeof(F)) Cplx {
  F re, im;
};

template <typename F>
__device__ __forceinline__ void store_cplx(F* p, F re, F im) {
  *reinterpret_cast<Cplx<F>*>(p) = Cplx<F>{re, im};
}

// Twiddles w_R^t = exp(-2 pi i t / R), t < R/2, for R = 2^B, computed in
// double precision and rounded once to the element's precision.
template <int S, int B, int NT>
__device__ __forceinline__ void make_twiddles(typename ComplexOf<S>::T* tw) {
  typedef typename ComplexOf<S>::T F;
  for (int t = (int)threadIdx.x; t < (1 << B) / 2; t += NT) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)(1 << B), &sn, &cs);
    tw[2 * t] = (F)cs;
    tw[2 * t + 1] = (F)sn;
  }
}

// Levels FIRST .. stages of the radix-2 DIT butterflies on `rows` staged rows
// of 2^b elements (a power of two: 2^b or 2^(b+1) for square tiles, fewer
// for rectangular ones): for blocks of 2^s, (a, b) -> (a + w^t b, a - w^t b),
// w = exp(-+ 2 pi i / 2^s) (sign + for the inverse).  Up to three levels run
// in one pass over LDS: levels s, s+1, s+2 as a radix-8 step on the eight
// elements t + j h (j < 8, h = 2^(s-1)) of a block of 2^(s+2), then a radix-4
// step (levels s, s+1 on t + j h, j < 4) and a radix-2 tail, so that L levels
// take ceil(L / 3) passes or one more.  Each step applies the same radix-2
// butterflies as level-by-level code; the twiddles come from the table, and
// a twiddle w_n^(p + n/4) = w_n^p * (-+ i) is applied exactly as that
// rotation.  A barrier ends each pass.  Lanes take consecutive rows at one
// butterfly position: with the padded row pitch their addresses are one
// element apart modulo the banks, free of conflicts at every level, and they
// read the same twiddle.  MAXR = 4 leaves out the radix-8 step (it holds
// eight complex values per thread).  The caller then writes the rows with tile_store
// (measured faster than storing the last pass's results directly: 16-byte
// row stores coalesce better than the butterflies' 8-byte element stores).
template <typename F>
__device__ __forceinline__ void bfly(F& ar, F& ai, F& br, F& bi, F wr, F wi) {
  const F tr = br * wr - bi * wi, ti = br * wi + bi * wr;
  br = ar - tr;
  bi = ai - ti;
  ar = ar + tr;
  ai = ai + ti;
}

// (r, i) * (-+ i): (i, -r) forward, (-i, r) inverse, exactly.
template <typename F>
__device__ __forceinline__ void rot_quarter(F wr, F wi, F sg, F* rr, F* ri) {
  *rr = sg * wi;
  *ri = -sg * wr;
}

template <int S, int B, int NT, int MAXR = 8, int FIRST = 1>
__device__ __forceinline__ void dit_rows(typename Bytes<S>::T* lds, int rows, int stages,
                                         bool inverse, const typename ComplexOf<S>::T* tw) {
  typedef typename ComplexOf<S>::T F;
  constexpr int R = 1 << B;
  constexpr int PE = TileShape<S, B, true>::PE;
  F* base = reinterpret_cast<F*>(lds);
  const F sg = inverse ? (F)-1 : (F)1;  // conjugates the forward twiddles
  const int rsh = 31 - __builtin_clz((unsigned)rows);  // rows is a power of two
  int s = FIRST;
  while (s <= stages) {
    const int h = 1 << (s - 1);
    if (MAXR >= 8 && s + 2 <= stages) {
      for (int beta = (int)threadIdx.x; beta < rows * (R / 8); beta += NT) {
        const int row = beta & (rows - 1);
        const int tp = beta >> rsh;
        const int t = tp & (h - 1);
        F* p = base + 2 * (row * PE + ((tp >> (s - 1)) << (s + 2)) + t);
        F xr[8], xi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          xr[j] = p[2 * j * h];
          xi[j] = p[2 * j * h + 1];
        }
        // level s: pairs (j, j+1), twiddle w_{2h}^t
        const F w1r = tw[2 * t * (R >> s)], w1i = sg * tw[2 * t * (R >> s) + 1];
#pragma unroll
        for (int j = 0; j < 8; j += 2) bfly(xr[j], xi[j], xr[j + 1], xi[j + 1], w1r, w1i);
        // level s+1: pairs (j, j+2), w_{4h}^t and w_{4h}^(t+h) = w_{4h}^t (-+ i)
        const F w2r = tw[2 * t * (R >> (s + 1))], w2i = sg * tw[2 * t * (R >> (s + 1)) + 1];
        F w2qr, w2qi;
        rot_quarter(w2r, w2i, sg, &w2qr, &w2qi);
        bfly(xr[0], xi[0], xr[2], xi[2], w2r, w2i);
        bfly(xr[4], xi[4], xr[6], xi[6], w2r, w2i);
        bfly(xr[1], xi[1], xr[3], xi[3], w2qr, w2qi);
        bfly(xr[5], xi[5], xr[7], xi[7], w2qr, w2qi);
        // level s+2: pairs (j, j+4), w_{8h}^(t+jh); j = 2, 3 are j = 0, 1
        // rotated by (-+ i)
        const int i3 = 2 * t * (R >> (s + 2)), i3h = 2 * (t + h) * (R >> (s + 2));
        const F w3r = tw[i3], w3i = sg * tw[i3 + 1];
        const F w4r = tw[i3h], w4i = sg * tw[i3h + 1];
        F w3qr, w3qi, w4qr, w4qi;
        rot_quarter(w3r, w3i, sg, &w3qr, &w3qi);
        rot_quarter(w4r, w4i, sg, &w4qr, &w4qi);
        bfly(xr[0], xi[0], xr[4], xi[4], w3r, w3i);
        bfly(xr[1], xi[1], xr[5], xi[5], w4r, w4i);
        bfly(xr[2], xi[2], xr[6], xi[6], w3qr, w3qi);
        bfly(xr[3], xi[3], xr[7], xi[7], w4qr, w4qi);
#pragma unroll
        for (int j = 0; j < 8; ++j) store_cplx(p + 2 * j * h, xr[j], xi[j]);
      }
      s += 3;
    } else if (s + 1 <= stages) {
      const int q4 = R >= 4 ? R / 4 : 1;  // R = 2 never gets here (stages <= b)
      for (int beta = (int)threadIdx.x; beta < rows * q4; beta += NT) {
        const int row = beta & (rows - 1);
        const int tp = beta >> rsh;
        const int t = tp & (h - 1);
        F* p = base + 2 * (row * PE + ((tp >> (s - 1)) << (s + 1)) + t);
        F xr[4], xi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          xr[j] = p[2 * j * h];
          xi[j] = p[2 * j * h + 1];
        }
        const F w1r = tw[2 * t * (R >> s)], w1i = sg * tw[2 * t * (R >> s) + 1];
        bfly(xr[0], xi[0], xr[1], xi[1], w1r, w1i);
        bfly(xr[2], xi[2], xr[3], xi[3], w1r, w1i);
        const F w2r = tw[2 * t * (R >> (s + 1))], w2i = sg * tw[2 * t * (R >> (s + 1)) + 1];
        F w2qr, w2qi;
        rot_quarter(w2r, w2i, sg, &w2qr, &w2qi);
        bfly(xr[0], xi[0], xr[2], xi[2], w2r, w2i);
        bfly(xr[1], xi[1], xr[3], xi[3], w2qr, w2qi);
#pragma unroll
        for (int j = 0; j < 4; ++j) store_cplx(p + 2 * j * h, xr[j], xi[j]);
      }
      s += 2;
    } else {
      for (int beta = (int)threadIdx.x; beta < rows * (R / 2); beta += NT) {
        const int row = beta & (rows - 1);
        const int tp = beta >> rsh;
        const int t = tp & (h - 1);
        F* pa = base + 2 * (row * PE + ((tp >> (s - 1)) << s) + t);
        F* pb = pa + 2 * h;
        F ar = pa[0], ai = pa[1], br = pb[0], bi = pb[1];
        bfly(ar, ai, br, bi, tw[2 * t * (R >> s)], sg * tw[2 * t * (R >> s) + 1]);
        store_cplx(pa, ar, ai);
        store_cplx(pb, br, bi);
      }
      s += 1;
    }
    __syncthreads();
  }
}

// The first levels of the DIT on values still in registers.  A tile thread
// whose PT = 2^p accesses cover rows x0 + i 2^(B-p) (i < PT) of one column
// holds, for each element of its chunks, the values that land on the 2^p
// consecutive destination positions rev_B(x) = rev_p(i) + 2^p rev_(B-p)(x0)
// of one destination row: a whole block of levels 1 .. p, whose twiddles
// w_2^0, w_4^{0,1} and w_8^{0..3} are constants (1, -+i and
// (+-1 -+ i)/sqrt 2).  Doing those levels here, between the loads and the
// scatter into LDS, saves dit_rows their passes over LDS (dit_rows then
// starts at level p + 1).  The arithmetic per butterfly is that of bfly.
template <int CPT, int CPR, int NT> constexpr int dit_reg_levels_of() {
  constexpr int PT = CPT / NT;
  return (CPT % NT != 0 || NT % CPR != 0 || PT < 2) ? 0 : (PT >= 8 ? 3 : (PT >= 4 ? 2 : 1));
}

template <typename F, int P, int LV>
__device__ __forceinline__ void dit_block_levels(F (&re)[P], F (&im)[P], F sg) {
  constexpr F C = (F)0.70710678118654752440084436210484904;
#pragma unroll
  for (int s = 1; s <= LV; ++s) {
    const int h = 1 << (s - 1);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (q & h) continue;
      const int t = q & (h - 1);  // twiddle w_{2h}^t
      const F br = re[q + h], bi = im[q + h];
      F tr, ti;
      if (t == 0) {
        tr = br;
        ti = bi;
      } else if (2 * t == h) {  // w = -+ i
        tr = sg * bi;
        ti = -sg * br;
      } else {  // h = 4, t = 1 or 3
        const F wr = t == 1 ? C : -C, wi = -sg * C;
        tr = br * wr - bi * wi;
        ti = br * wi + bi * wr;
      }
      re[q + h] = re[q] - tr;
      im[q + h] = im[q] - ti;
      re[q] = re[q] + tr;
      im[q] = im[q] + ti;
    }
  }
}

// Levels 1 .. LV (LV <= p = log2 PT <= 3; see above) on a thread's chunks,
// in place: chunk i keeps row x0 + i 2^(B-p).
template <int S, int VB, int PT, int LV>
__device__ __forceinline__ void dit_reg_levels_n(Chunk<S, VB> (&reg)[PT], bool inverse) {
  typedef typename ComplexOf<S>::T F;
  static_assert(PT == 2 || PT == 4 || PT == 8, "two, four or eight rows per thread");
  constexpr int p = PT == 8 ? 3 : (PT == 4 ? 2 : 1);
  static_assert(LV >= 1 && LV <= p, "levels held by the thread's rows");
  constexpr int CE = VB / S;
  const F sg = inverse ? (F)-1 : (F)1;
#pragma unroll
  for (int e = 0; e < CE; ++e) {
    F re[PT], im[PT];
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      Cplx<F> c;
      __builtin_memcpy(&c, &reg[crev(q, p)].e[e], sizeof(c));
      re[q] = c.re;
      im[q] = c.im;
    }
    dit_block_levels<F, PT, LV>(re, im, sg);
#pragma unroll
    for (int q = 0; q < PT; ++q) {
      const Cplx<F> c{re[q], im[q]};
      __builtin_memcpy(&reg[crev(q, p)].e[e], &c, sizeof(c));
    }
  }
}

// LDS passes dit_rows makes for `levels` levels: radix 8 (MAXR 8) while
// three or more remain, then radix 4, then radix 2.
__host__ __device__ constexpr int dit_passes(int levels, int maxr) {
  int p = 0;
  while (levels > 0) {
    levels -= (maxr >= 8 && levels >= 3) ? 3 : (levels >= 2 ? 2 : 1);
    ++p;
  }
  return p;
}

// Whether the first PRE levels go to registers: only where that saves
// dit_rows a pass over LDS (at five levels, radix 8 + 4 after none and
// 4 + 4 after one are both two passes, and the radix-8 form measured 1%
// faster).
__host__ __device__ constexpr bool dit_pre_pays(int stages, int pre, int maxr) {
  return pre > 0 && stages >= pre && dit_passes(stages - pre, maxr) < dit_passes(stages, maxr);
}

// Levels 1 .. log2 PT on a thread's chunks when `apply` (uniform).
template <int S, int VB, int PT>
__device__ __forceinline__ void dit_reg_levels(Chunk<S, VB> (&reg)[PT], bool apply, bool inverse) {
  constexpr int p = PT == 8 ? 3 : (PT == 4 ? 2 : 1);
  if (apply) dit_reg_levels_n<S, VB, PT, p>(reg, inverse);
}

// dit_rows from level 1, or from level PRE + 1 after the register levels
// (the first level a compile-time constant either way: a run-time first
// level cost the two-tile kernels 1% at three and five levels).
template <int S, int B, int NT, int MAXR, int PRE>
__device__ __forceinline__ void dit_rows_after(typename Bytes<S>::T* lds, int rows, int stages,
                                               bool inverse, const typename ComplexOf<S>::T* tw,
                                               bool pre) {
  if constexpr (PRE > 0) {
    if (pre) return dit_rows<S, B, NT, MAXR, PRE + 1>(lds, rows, stages, inverse, tw);
  }
  dit_rows<S, B, NT, MAXR, 1>(lds, rows, stages, inverse, tw);
}

// ---------------------------------------------------------------------------
// In-place square transpose (the middle step of the paper's recursive
// method, Methods): a 2^h x 2^h matrix in 2^b x 2^b tiles; tiles (R, C) and
// (C, R) swap through LDS, each transposed; diagonal tiles transpose alone.
// ---------------------------------------------------------------------------

// The w-th pair (R, C) with R <= C, column by column: C = c holds
// R = 0 .. c, so pairs before column c number c (c + 1) / 2.
__host__ __device__ __forceinline__ void tri_pair(uint64_t w, uint32_t* r, uint32_t* c) {
  uint64_t cc = (uint64_t)((__builtin_sqrt(8.0 * (double)w + 1.0) - 1.0) * 0.5);
  while ((cc + 1) * (cc + 2) / 2 <= w) ++cc;
  while (cc * (cc + 1) / 2 > w) --cc;
  *c = (uint32_t)cc;
  *r = (uint32_t)(w - cc * (cc + 1) / 2);
}

template <int S, int B, bool VEC, int NT>
__device__ __forceinline__ void tile_pair_transpose(typename Bytes<S>::T* __restrict__ base, int h,
                                                    uint32_t tr, uint32_t tc,
                                                    typename Bytes<S>::T* lds) {
  typedef TileShape<S, B, VEC> Sh;
  constexpr int PT = (Sh::CPT + NT - 1) / NT;
  const uint64_t rowstride = 1ull << h;
  // tile (R, C) starts at row R 2^b, column C 2^b; tile_load's "y" selects
  // the column block, so pass the row block through the base pointer
  typename Bytes<S>::T* a = base + ((uint64_t)tr << (B + h));
  typename Bytes<S>::T* b = base + ((uint64_t)tc << (B + h));
  const bool diag = (tr == tc);
  Chunk<S, Sh::VB> ra[PT], rb[PT];
  tile_load<S, B, VEC, NT, PT>(ra, a, rowstride, tc);
  if (!diag) tile_load<S, B, VEC, NT, PT>(rb, b, rowstride, tr);
  tile_scatter<S, B, VEC, NT, PT, 0>(ra, lds);
  if (!diag) tile_scatter<S, B, VEC, NT, PT, 0>(rb, lds + Sh::TILE_E);
  __syncthreads();
  tile_store<S, B, VEC, NT, PT>(b, rowstride, tr, lds);
  if (!diag) tile_store<S, B, VEC, NT, PT>(a, rowstride, tc, lds + Sh::TILE_E);
}

// ---------------------------------------------------------------------------
// Whole array in one workgroup's LDS (any 2^k that fits): load, barrier,
// out[i] = lds[rev_k(i)].  One element per access; the padding of one
// element every 32 breaks the power-of-two strides of the gather.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t small_slot(uint32_t i) { return i + (i >> 5); }

template <int S, int NT>
__device__ __forceinline__ void small_array(const typename Bytes<S>::T* src,
                                            typename Bytes<S>::T* dst, int k,
                                            typename Bytes<S>::T* lds) {
  const uint32_t n = 1u << k;
  for (uint32_t i = threadIdx.x; i < n; i += NT) lds[small_slot(i)] = src[i];
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += NT) dst[i] = lds[small_slot(rev_bits(i, k))];
}

// ---------------------------------------------------------------------------
// Whole array in one wavefront (n = 2^k <= 64): lane i holds element i and
// fetches element rev_k(i) from its lane with ds_bpermute, one dword at a
// time.  No LDS storage and no barrier.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ void wave_array(const typename Bytes<S>::T* src,
                                           typename Bytes<S>::T* dst, int k, int lane,
                                           int digit = 1) {
  typedef typename Bytes<S>::T E;
  const int n = 1 << k;
  const bool live = lane < n;
  const int from = (int)(digit == 1 ? rev_bits((uint32_t)lane, k)
                                    : drev_bits((uint32_t)lane & ((1u << k) - 1u), k, digit)) * 4;
  E v;
  if constexpr (S <= 4) {
    v = live ? src[lane] : (E)0;
    const uint32_t w = __builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)v);
    if (live) dst[lane] = (E)w;
  } else {
    if (live) {
      v = src[lane];
    } else {
      v = (E)0u;
    }
    E out;
#pragma unroll
    for (int d = 0; d < S / 4; ++d) out[d] = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)v[d]);
    if (live) dst[lane] = out;
  }
}

}  // namespace bitrev
