// The C ABI of libbitrev: argument validation (before any HIP call), the
// plan (which path, tile width, grid), the tuning table, and the launches.
#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <tuple>

#include "bitrev.h"
#include "bitrev_device.hpp"
#include "bitrev_launch.hpp"

namespace {

using namespace bitrev;

thread_local int g_last_hip_error = 0;

bitrev_status_t hip_fail(hipError_t e) {
  g_last_hip_error = (int)e;
  return BITREV_ERROR_HIP;
}

// ---------------------------------------------------------------------------
// Device properties (cached per device).
// ---------------------------------------------------------------------------
struct DeviceInfo {
  int cus = 256;                 // compute units
  size_t lds_per_block = 163840; // LDS bytes a workgroup may use
  int xcds = 8;                  // XCDs the dispatcher deals workgroups over
};

constexpr int kMaxDevices = 64;
std::mutex g_dev_mu;
bool g_dev_known[kMaxDevices];
DeviceInfo g_dev[kMaxDevices];

// The current device's properties; MI355X figures when `allow_default` and
// no device is present (plan queries on a host without a GPU).
bitrev_status_t device_info(DeviceInfo* out, bool allow_default, bool* present = nullptr) {
  int dev = 0;
  if (present) *present = false;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    if (allow_default) {
      (void)hipGetLastError();
      *out = DeviceInfo();
      return BITREV_SUCCESS;
    }
    return hip_fail(e != hipSuccess ? e : hipErrorInvalidDevice);
  }
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if (!g_dev_known[dev]) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return hip_fail(e);
    DeviceInfo d;
    d.cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 1;
    d.lds_per_block = p.sharedMemPerBlock;
    // gfx950 has 32 compute units per XCD; a partitioned device shows fewer.
    int x = (d.cus + 16) / 32;
    if (strncmp(p.gcnArchName, "gfx942", 6) == 0) x = (d.cus + 19) / 38;
    if (x < 1) x = 1;
    if (const char* env = getenv("BITREV_XCDS")) {
      const int v = atoi(env);
      if (v >= 1 && v <= 64) x = v;
    }
    d.xcds = x;
    g_dev[dev] = d;
    g_dev_known[dev] = true;
  }
  *out = g_dev[dev];
  if (present) *present = true;
  return BITREV_SUCCESS;
}

// ---------------------------------------------------------------------------
// Tuning table: (mode, elem_size, log2n or -1) -> tile bits, workgroups per
// CU, order.  Loaded from a text file; the built-in defaults apply otherwise.
// ---------------------------------------------------------------------------
struct TuneEntry {
  int tile_bits = 0;
  int wg_per_cu = 0;
  int order = 0;
  int variant = 0;
  int xcd_remap = 0;
  int cache_hints = 0;
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, TuneEntry> g_tune;
std::once_flag g_tune_env_once;

const char kTuningFormat[] =
    "libbitrev tuning v2: one entry per line, '#' starts a comment; fields: mode "
    "(inplace|outofplace|batched) elem_size log2n(-1 = any) tile_bits(0 = default) "
    "wg_per_cu(0 = default) order(0 = default, 1 natural, 2 balanced, 3 grouped) "
    "variant(0 = default, 1 one item per workgroup, 2 persistent pipelined, 3 register-staged) "
    "xcd_remap(0 = default, 1 contiguous ranges per XCD, 2 dispatch order) "
    "[cache_hints(0 = default, 1 plain, 2 streaming loads, 3 streaming stores, "
    "4 streaming loads and write-through stores)]";

int mode_from_name(const char* s) {
  if (strcmp(s, "inplace") == 0) return 0;
  if (strcmp(s, "outofplace") == 0) return 1;
  if (strcmp(s, "batched") == 0) return 2;
  return -1;
}

bool valid_elem_size(size_t s) { return s == 1 || s == 2 || s == 4 || s == 8 || s == 16; }

bitrev_status_t load_tuning_file(const char* path) {
  if (path == NULL) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return BITREV_SUCCESS;
  }
  FILE* f = fopen(path, "r");
  if (!f) return BITREV_ERROR_INVALID_VALUE;
  std::map<std::tuple<int, int, int>, TuneEntry> table;
  char line[512];
  bool ok = true;
  while (fgets(line, sizeof line, f)) {
    char* hash = strchr(line, '#');
    if (hash) *hash = '\0';
    char mode[32];
    int s, k, b, wg, order, variant, xcd, hints = 0;
    char extra[8];
    const int got = sscanf(line, "%31s %d %d %d %d %d %d %d %d %7s", mode, &s, &k, &b, &wg,
                           &order, &variant, &xcd, &hints, extra);
    if (got <= 0) continue;  // blank or comment-only line
    const int md = got >= 8 ? mode_from_name(mode) : -1;
    if ((got != 8 && got != 9) || md < 0 || !valid_elem_size((size_t)s) || k < -1 ||
        k > BITREV_MAX_LOG2N || b < 0 || b > kMaxTileBits || wg < 0 || wg > 1024 || order < 0 ||
        order > 3 || variant < 0 || variant > 3 || xcd < 0 || xcd > 2 || hints < 0 || hints > 4) {
      ok = false;
      break;
    }
    TuneEntry t;
    t.tile_bits = b;
    t.wg_per_cu = wg;
    t.order = order;
    t.variant = variant;
    t.xcd_remap = xcd;
    t.cache_hints = hints;
    table[std::make_tuple(md, s, k)] = t;
  }
  fclose(f);
  if (!ok) return BITREV_ERROR_INVALID_VALUE;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.swap(table);
  return BITREV_SUCCESS;
}

void load_env_tuning() {
  std::call_once(g_tune_env_once, [] {
    const char* p = getenv("BITREV_TUNING_FILE");
    if (p && *p) (void)load_tuning_file(p);
  });
}

TuneEntry tune_lookup(int mode, int s, int k) {
  load_env_tuning();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(mode, s, k));
  if (it == g_tune.end()) it = g_tune.find(std::make_tuple(mode, s, -1));
  return it == g_tune.end() ? TuneEntry() : it->second;
}

// ---------------------------------------------------------------------------
// Plans.
// ---------------------------------------------------------------------------
enum { kModeInplace = 0, kModeOutofplace = 1, kModeBatched = 2 };

// Built-in plan per (mode, element size, array bytes), from sweeps of tile
// width x work order x kernel variant x XCD renumbering on MI355X with the
// caches evicted before each call (arrays of 8 MiB to 4 GiB); each entry is
// the one closest to the best at every measured size of its class.  Rows of
// 2^b * s >= 128 bytes keep every HBM access a run of whole 128-byte lines.
// "small" arrays (<= 512 MiB) interact with the 256 MiB Infinity Cache and
// favour different choices than arrays far beyond it.  The cache hints are
// chosen separately (default_hints).
struct DefaultPlan {
  int b;
  int variant;   // 1 one item per workgroup, 2 persistent pipelined, 3 register-staged
  int order;     // 1 natural, 2 balanced, 3 grouped
  int xcd_remap; // 1 contiguous ranges per XCD, 2 dispatch order
  int wg_per_cu = 0;  // batched: persistent workgroups per CU (0 = as many as fit)
};

DefaultPlan default_plan(int mode, int s, uint64_t array_bytes) {
  const bool small = array_bytes <= (512ull << 20);
  // up to 32 MiB the launch is short and the persistent pipelined kernel
  // in dispatch order does best (complex64: within 2% of the best plan)
  const bool tiny = array_bytes > 0 && array_bytes <= (32ull << 20);
  if (tiny && mode == 0) return {s >= 16 ? 5 : (s == 8 ? 5 : (s == 4 ? 6 : 7)), 2, 1, 2};
  if (tiny && mode == 1) return {s >= 8 ? 5 : (s == 4 ? 6 : 7), 2, s == 8 ? 3 : 2, 2};
  if (mode == 0) {  // in place
    // the grouped order keeps runs of neighbouring tiles on both sides of
    // each swap: complex64 2^24 +8%, float32 256 MiB +30%, complex128
    // 64 MiB +13%, int16 +1%; where it measured slower (float32 up to
    // 64 MiB, complex128 128-512 MiB: -3%) the balanced order stays
    const bool mid = array_bytes > (64ull << 20);
    switch (s) {
      case 1: return {7, 1, 2, small ? 2 : 1};
      case 2: return {7, 1, 3, 2};
      case 4: return mid ? DefaultPlan{6, 1, 3, 2} : DefaultPlan{6, 2, 2, 1};
      // complex64 above 64 MiB up to 128 MiB: b = 5 in natural order with
      // write-through stores (2^24: 5816 -> 5990 GB/s per call, ranges
      // apart over eight alternating rounds; it loses 3-12% from 256 MiB up)
      case 8: return (array_bytes > (64ull << 20) && array_bytes <= (128ull << 20))
                         ? DefaultPlan{5, 1, 1, 2}
                         : DefaultPlan{6, 1, 3, 2};
      default:
        // complex128 of 128-512 MiB: the register-staged kernel (twice the
        // pairs in flight), balanced up to 256 MiB, grouped at 512 MiB
        // (+1%, +2.6%, +7% over the one-item plans)
        if (!mid || !small) return {5, 1, 3, 2};
        return array_bytes <= (256ull << 20) ? DefaultPlan{5, 3, 2, 2} : DefaultPlan{5, 3, 3, 2};
    }
  }
  if (mode == 2) {  // batched (in place, persistent): complex64 measured on 4096 uneven arrays
    switch (s) {
      // complex64: one 1024-thread workgroup per CU; two fit (62 VGPRs,
      // 65 KiB of LDS each) but measured 4.5% slower on the 4096-array batch
      case 8: return {6, 0, 1, 1, 1};
      case 16: return {5, 0, 2, 1};
      default: return {default_plan(0, s, 0).b, 0, 2, 1};
    }
  }
  switch (s) {  // out of place
    // 1 and 2 bytes: natural order in dispatch order (uint8 2^26-2^28: +15%)
    case 1: return {7, 1, 1, 2};
    case 2: return {7, 1, 1, 2};
    case 4: return small ? DefaultPlan{6, 1, 1, 2} : DefaultPlan{6, 1, 2, 1};
    case 8: return {5, 1, 2, 1};
    default: return {5, 1, 2, 1};
  }
}


int occupancy_of(int s, int b, bool vec, bool inplace, bool pipelined) {
  switch (s) {
    case 1: return tile_occupancy_s1(b, vec, inplace, pipelined);
    case 2: return tile_occupancy_s2(b, vec, inplace, pipelined);
    case 4: return tile_occupancy_s4(b, vec, inplace, pipelined);
    case 8: return tile_occupancy_s8(b, vec, inplace, pipelined);
    default: return tile_occupancy_s16(b, vec, inplace, pipelined);
  }
}

int rs_threads_of(int s, int b, bool vec) {
  switch (s) {
    case 1: return tile_rs_threads_s1(b, vec);
    case 2: return tile_rs_threads_s2(b, vec);
    case 4: return tile_rs_threads_s4(b, vec);
    case 8: return tile_rs_threads_s8(b, vec);
    default: return tile_rs_threads_s16(b, vec);
  }
}

int threads_of(int s, int b, bool vec) {
  switch (s) {
    case 1: return tile_threads_s1(b, vec);
    case 2: return tile_threads_s2(b, vec);
    case 4: return tile_threads_s4(b, vec);
    case 8: return tile_threads_s8(b, vec);
    default: return tile_threads_s16(b, vec);
  }
}

#ifndef BITREV_GROUP_J
#define BITREV_GROUP_J 3
#endif

// The kernels' order code (bit 0 balanced, bits 1.. group width) for a
// plan's order: 1 natural, 2 balanced, 3 grouped.
int order_code(int order) {
  // grouped: groups in pair_at's natural order (measured 1% ahead of the
  // balanced group order for complex64 2^24-2^26); the kernels clamp j
  if (order == 3) return BITREV_GROUP_J << 1;
  return order == 2 ? 1 : 0;
}

bool valid_config(const bitrev_config_t* c) {
  if (!c) return true;
  return c->tile_bits >= 0 && c->tile_bits <= kMaxTileBits && c->grid_blocks >= 0 &&
         c->order >= 0 && c->order <= 3 && c->variant >= 0 && c->variant <= 3 &&
         c->xcd_remap >= 0 && c->xcd_remap <= 2 && c->cache_hints >= 0 && c->cache_hints <= 4;
}

uint32_t round_up(uint64_t v, uint32_t to) {
  const uint64_t r = (v + to - 1) / to * to;
  return (uint32_t)(r > 0xFFFFFFFFull ? 0xFFFFFFFFull / to * to : r);
}

// Grid for `items` work items: one workgroup per item up to 2^20
// workgroups (then a grid-stride loop), a multiple of the XCD count.
uint32_t default_grid(uint64_t items, const DeviceInfo& d) {
  const uint64_t cap = 1ull << 20;
  return round_up(items < cap ? items : cap, (uint32_t)d.xcds);
}

int resident_per_cu(int threads, size_t lds);

// The Infinity Cache of MI355X: arrays beyond it stream through HBM.
constexpr uint64_t kCacheBytes = 256ull << 20;

// Cache hints of the built-in plans, from sweeps over element sizes (1-16
// bytes) and array sizes (64 MiB - 4 GiB) on random data.  Streaming loads
// with write-through stores were the best or tied form almost everywhere:
// complex64 in place +4.5% at 64 MiB and +7.7% at 256 MiB over streaming
// stores; out of place +3-6%; complex128 and float32 +1-5%; complex64 in
// place at 128 MiB on its b = 5 plan +13% over streaming stores.  Streaming
// loads alone
// stay where they measured ahead: 1- and 2-byte elements beyond the Infinity
// Cache (out of place +15%) and float32 out of place at 256 MiB (+4%).
// Below 32 MiB (out of place) or 64 MiB (in place) accesses stay plain.
int default_hints(int mode, int s, uint64_t array_bytes, int64_t rows) {
  const uint64_t total = array_bytes * (uint64_t)(rows > 0 ? rows : 1);
  if (total < (mode == kModeInplace ? (64ull << 20) : (32ull << 20))) return kHintPlain;
  if (s <= 2 && total > kCacheBytes) return kHintStreamLoads;
  if (mode != kModeInplace && s == 4 && total > (128ull << 20) && total <= kCacheBytes)
    return kHintStreamLoads;
  return kHintStreamWriteThrough;
}

struct Plan {
  int path = BITREV_PATH_NONE;
  int b = 0;
  int m = 0;
  int threads = 0;
  uint32_t grid = 0;
  int order = 2;
  int variant = 1;
  int xcd_remap = 1;
  int hints = kHintPlain;  // CacheHint of the one-item 16-byte tile kernels
  bool vec = true;
  uint64_t items_per_seg = 0;
  uint64_t total = 0;
  size_t lds = 0;
};

// Plan for a plain call (mode 0 or 1) on `rows` arrays of 2^k elements.
// align: the largest power of two (<= 16) dividing both data pointers.
bitrev_status_t plan_plain(int mode, int k, int s, int64_t rows, const bitrev_config_t* cfg,
                           size_t align, const DeviceInfo& d, bool have_device, Plan* p) {
  *p = Plan();
  if (rows == 0 || (mode == kModeInplace && k <= 1)) return BITREV_SUCCESS;
  const int forced_b = cfg ? cfg->tile_bits : 0;
  const TuneEntry te = tune_lookup(mode, s, k);
  // the size class is the launch's whole footprint: 256 rows of 2^16 float32
  // (64 MiB) run 15% faster on the 64 MiB plan than on the plan of one
  // 256 KiB row
  const uint64_t row_bytes = ((uint64_t)s) << k;
  const uint64_t rows_u = rows > 0 ? (uint64_t)rows : 1u;
  const uint64_t footprint = row_bytes > UINT64_MAX / rows_u ? UINT64_MAX : row_bytes * rows_u;
  const DefaultPlan dp = default_plan(mode, s, footprint);
  p->order = (cfg && cfg->order) ? cfg->order : (te.order ? te.order : dp.order);
  p->xcd_remap = (cfg && cfg->xcd_remap) ? cfg->xcd_remap
                                         : (te.xcd_remap ? te.xcd_remap : dp.xcd_remap);
  if (forced_b == 0 && k <= 6) {
    p->path = BITREV_PATH_WAVE;
    p->threads = 256;
    const uint64_t wg = ((uint64_t)rows + 3) / 4;
    p->grid = (uint32_t)(wg < 65536 ? wg : 65536);
    if (cfg && cfg->grid_blocks > 0) p->grid = (uint32_t)cfg->grid_blocks;
    p->total = (uint64_t)rows;
    return BITREV_SUCCESS;
  }
  p->variant = (cfg && cfg->variant) ? cfg->variant : (te.variant ? te.variant : dp.variant);
  if (p->variant == 3 && mode != kModeInplace) p->variant = 1;  // register staging is in place only
  // LDS tiles per workgroup: a pair in place (one when register-staged)
  const int inplace_tiles = (mode == kModeInplace && p->variant != 3) ? 2 : 1;
  int b;
  if (forced_b > 0) {
    b = forced_b;
    if (2 * b > k || b > max_tile_bits(s) ||
        tile_lds_bytes_for(s, b, inplace_tiles) > d.lds_per_block)
      return BITREV_ERROR_NOT_SUPPORTED;
  } else {
    b = te.tile_bits ? te.tile_bits : dp.b;
    if (b > max_tile_bits(s)) b = max_tile_bits(s);
    if (2 * b > k) b = k / 2;
    while (b > 0 && tile_lds_bytes_for(s, b, inplace_tiles) > d.lds_per_block) --b;
  }
  const int m = k - 2 * b;
  if (m > 32) return BITREV_ERROR_NOT_SUPPORTED;
  const size_t vb = ((size_t)s << b) < 16 ? ((size_t)s << b) : 16;
  p->vec = (align % vb) == 0;
  p->path = BITREV_PATH_TILE;
  p->b = b;
  p->m = m;
  p->items_per_seg = (mode == kModeInplace) ? pair_count(m) : (1ull << m);
  if ((uint64_t)rows > (1ull << 62) / p->items_per_seg) return BITREV_ERROR_NOT_SUPPORTED;
  p->total = p->items_per_seg * (uint64_t)rows;
  p->threads = p->variant == 3 ? rs_threads_of(s, b, p->vec) : threads_of(s, b, p->vec);
  p->lds = tile_lds_bytes_for(s, b, inplace_tiles);
  p->hints = (cfg && cfg->cache_hints)
                 ? cfg->cache_hints - 1
                 : (te.cache_hints ? te.cache_hints - 1 : default_hints(mode, s, (uint64_t)s << k, rows));
  if (cfg && cfg->grid_blocks > 0) {
    p->grid = round_up((uint64_t)cfg->grid_blocks, (uint32_t)d.xcds);
  } else if (te.wg_per_cu > 0) {
    p->grid = round_up((uint64_t)te.wg_per_cu * d.cus, (uint32_t)d.xcds);
  } else if (p->variant == 2) {
    // persistent: the workgroups that are resident at once
    int occ = have_device ? occupancy_of(s, b, p->vec, mode == kModeInplace, true) : 0;
    if (occ <= 0) occ = resident_per_cu(p->threads, p->lds);
    const uint64_t g = (uint64_t)occ * d.cus;
    p->grid = round_up(g < p->total ? g : p->total, (uint32_t)d.xcds);
  } else {
    p->grid = default_grid(p->total, d);
  }
  return BITREV_SUCCESS;
}

// Workgroups of the batched kernel that fit on one CU at once: limited by
// LDS (160 KiB per CU) and by 32 wavefronts per CU.
int resident_per_cu(int threads, size_t lds) {
  const int by_waves = 32 / ((threads + 63) / 64);
  const int by_lds = lds ? (int)(163840 / lds) : by_waves;
  const int r = by_waves < by_lds ? by_waves : by_lds;
  return r < 1 ? 1 : r;
}

int batched_occupancy_of(int s, int b, bool oop) {
  switch (s) {
    case 1: return batched_occupancy_s1(b, oop);
    case 2: return batched_occupancy_s2(b, oop);
    case 4: return batched_occupancy_s4(b, oop);
    case 8: return batched_occupancy_s8(b, oop);
    default: return batched_occupancy_s16(b, oop);
  }
}

bitrev_status_t plan_batched(int s, const bitrev_config_t* cfg, const DeviceInfo& d,
                             bool have_device, bool oop, Plan* p) {
  *p = Plan();
  const TuneEntry te = tune_lookup(kModeBatched, s, -1);
  const DefaultPlan dp = default_plan(kModeBatched, s, 0);
  int b = (cfg && cfg->tile_bits) ? cfg->tile_bits : (te.tile_bits ? te.tile_bits : dp.b);
  if (!(cfg && cfg->tile_bits) && b > max_tile_bits(s)) b = max_tile_bits(s);
  if (b < kMinBatchedTileBits || b > max_tile_bits(s) ||
      tile_lds_bytes_for(s, b, 2) > d.lds_per_block)
    return BITREV_ERROR_NOT_SUPPORTED;
  p->path = BITREV_PATH_BATCHED;
  p->b = b;
  p->order = (cfg && cfg->order) ? cfg->order : (te.order ? te.order : dp.order);
  // out of place, complex64 (4096 arrays of 2^8-2^20): eight workgroups per
  // CU in dispatch order, 4338 -> 5246 GB/s over the in-place choice (one per
  // CU, contiguous XCD ranges); two or four per CU came within 1%
  const bool oop_c64 = oop && s == 8 && b == dp.b;
  p->xcd_remap = (cfg && cfg->xcd_remap) ? cfg->xcd_remap
                                         : (te.xcd_remap ? te.xcd_remap
                                                         : (oop_c64 ? 2 : dp.xcd_remap));
  p->threads = threads_of(s, b, true);
  p->lds = tile_lds_bytes_for(s, b, 2);
  int per_cu = te.wg_per_cu;
  // the built-in count belongs to the built-in tile width only
  if (per_cu <= 0 && b == dp.b) per_cu = oop_c64 ? 8 : dp.wg_per_cu;
  if (per_cu <= 0) {
    // resident at once: LDS and threads, and the registers the kernel needs
    per_cu = resident_per_cu(p->threads, p->lds);
    const int occ = have_device ? batched_occupancy_of(s, b, oop) : 0;
    if (occ > 0 && occ < per_cu) per_cu = occ;
  }
  if (cfg && cfg->grid_blocks > 0) {
    p->grid = round_up((uint64_t)cfg->grid_blocks, (uint32_t)d.xcds);
  } else {
    p->grid = round_up((uint64_t)per_cu * d.cus, (uint32_t)d.xcds);
  }
  return BITREV_SUCCESS;
}

// ---------------------------------------------------------------------------
// Launches.
// ---------------------------------------------------------------------------
hipError_t launch_tile(bool inplace, int s, const Plan& p, const void* src, void* dst,
                       uint64_t src_stride, uint64_t dst_stride, const DeviceInfo& d,
                       hipStream_t st, void* ev_start = nullptr, void* ev_stop = nullptr) {
  TileLaunch a;
  a.ev_start = ev_start;
  a.ev_stop = ev_stop;
  a.src = src;
  a.dst = dst;
  a.m = p.m;
  a.items_per_seg = p.items_per_seg;
  a.total_items = p.total;
  a.seg_elems = src_stride;
  a.dst_seg_elems = dst_stride;
  a.balanced = order_code(p.order);
  a.xcds = p.xcd_remap == 2 ? 1 : d.xcds;
  a.grid = p.grid;
  a.pipelined = p.variant == 2 ? 1 : (p.variant == 3 ? 2 : 0);
  a.hints = p.hints;
  switch (s) {
    case 1: return inplace ? launch_tile_inplace_s1(p.b, p.vec, a, st) : launch_tile_outofplace_s1(p.b, p.vec, a, st);
    case 2: return inplace ? launch_tile_inplace_s2(p.b, p.vec, a, st) : launch_tile_outofplace_s2(p.b, p.vec, a, st);
    case 4: return inplace ? launch_tile_inplace_s4(p.b, p.vec, a, st) : launch_tile_outofplace_s4(p.b, p.vec, a, st);
    case 8: return inplace ? launch_tile_inplace_s8(p.b, p.vec, a, st) : launch_tile_outofplace_s8(p.b, p.vec, a, st);
    default: return inplace ? launch_tile_inplace_s16(p.b, p.vec, a, st) : launch_tile_outofplace_s16(p.b, p.vec, a, st);
  }
}

hipError_t launch_wave(int s, const Plan& p, const void* src, void* dst, int k, int64_t rows,
                       uint64_t src_stride, uint64_t dst_stride, hipStream_t st) {
  WaveLaunch a;
  a.src = src;
  a.dst = dst;
  a.k = k;
  a.nseg = (uint64_t)rows;
  a.grid = p.grid;
  a.src_stride = src_stride;
  a.dst_stride = dst_stride;
  switch (s) {
    case 1: return launch_wave_s1(a, st);
    case 2: return launch_wave_s2(a, st);
    case 4: return launch_wave_s4(a, st);
    case 8: return launch_wave_s8(a, st);
    default: return launch_wave_s16(a, st);
  }
}

size_t pointer_align(const void* a, const void* b) {
  const uintptr_t v = reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b);
  size_t al = 16;
  while (al > 1 && (v & (al - 1))) al >>= 1;
  return al;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

// Common body of bitrev_inplace/outofplace/rows (+ _ex).
// Largest power of two <= 16 dividing v (16 for v = 0).
size_t align_of(uint64_t v) {
  size_t al = 16;
  while (al > 1 && (v & (al - 1))) al >>= 1;
  return al;
}

// Bytes spanned by `rows` arrays of n elements placed `stride` elements apart.
uint64_t footprint(uint64_t n, int64_t rows, uint64_t stride, size_t s) {
  return rows <= 0 ? 0 : ((uint64_t)(rows - 1) * stride + n) * s;
}

bool ranges_overlap(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bbytes && y < x + abytes;
}

// Common body of the plain, rows and strided entry points.  Strides are in
// elements between consecutive arrays; 0 means 2^k (contiguous rows).
// ev_start / ev_stop: optional hipEvent_t recorded as the path's one kernel
// starts and ends (around the launch where the path is not a tile kernel).
bitrev_status_t run_plain(const void* src, void* dst, int k, int64_t rows, size_t s,
                          const bitrev_config_t* cfg, void* stream, uint64_t src_stride = 0,
                          uint64_t dst_stride = 0, void* ev_start = nullptr,
                          void* ev_stop = nullptr) {
  // ---- validation: no HIP call before this block completes ----
  if (src == NULL || dst == NULL) return BITREV_ERROR_INVALID_VALUE;
  if (k < 0 || k > BITREV_MAX_LOG2N || !valid_elem_size(s) || rows < 0 || !valid_config(cfg))
    return BITREV_ERROR_INVALID_VALUE;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % s)
    return BITREV_ERROR_INVALID_VALUE;
  const uint64_t n = 1ull << k;
  if (src_stride == 0) src_stride = n;
  if (dst_stride == 0) dst_stride = n;
  if (src_stride < n || dst_stride < n || src_stride > (1ull << 50) || dst_stride > (1ull << 50))
    return BITREV_ERROR_INVALID_VALUE;
  if (rows > 0 && ((uint64_t)rows > (1ull << 62) / (src_stride * s) ||
                   (uint64_t)rows > (1ull << 62) / (dst_stride * s)))
    return BITREV_ERROR_INVALID_VALUE;
  const bool inplace = (src == dst);
  if (inplace && src_stride != dst_stride) return BITREV_ERROR_INVALID_VALUE;
  if (!inplace && ranges_overlap(src, footprint(n, rows, src_stride, s), dst,
                                 footprint(n, rows, dst_stride, s)))
    return BITREV_ERROR_ALIAS;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const bool timed = ev_start != nullptr && ev_stop != nullptr;
  if (rows == 0 || (inplace && k <= 1)) {
    if (!timed) return BITREV_SUCCESS;  // nothing to run: the events bracket nothing
    hipError_t e = hipEventRecord(static_cast<hipEvent_t>(ev_start), hs);
    if (e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(ev_stop), hs);
    return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
  }
  // ---- plan and launch ----
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  Plan p;
  size_t align = pointer_align(src, dst);
  if (rows > 1) {
    const size_t sa = align_of(src_stride * s), da = align_of(dst_stride * s);
    if (sa < align) align = sa;
    if (da < align) align = da;
  }
  st = plan_plain(inplace ? kModeInplace : kModeOutofplace, k, (int)s, rows, cfg, align, d, true,
                  &p);
  if (st != BITREV_SUCCESS) return st;
  hipError_t e = hipSuccess;
  if (p.path == BITREV_PATH_WAVE) {
    if (timed) e = hipEventRecord(static_cast<hipEvent_t>(ev_start), hs);
    if (e == hipSuccess) e = launch_wave((int)s, p, src, dst, k, rows, src_stride, dst_stride, hs);
    if (timed && e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(ev_stop), hs);
  } else if (p.path == BITREV_PATH_TILE) {
    e = launch_tile(inplace, (int)s, p, src, dst, src_stride, dst_stride, d, hs,
                    timed ? ev_start : nullptr, timed ? ev_stop : nullptr);
  }
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

hipError_t launch_transpose(int s, int b, bool vec, const TransposeLaunch& a, hipStream_t st) {
  switch (s) {
    case 1: return launch_transpose_s1(b, vec, a, st);
    case 2: return launch_transpose_s2(b, vec, a, st);
    case 4: return launch_transpose_s4(b, vec, a, st);
    case 8: return launch_transpose_s8(b, vec, a, st);
    default: return launch_transpose_s16(b, vec, a, st);
  }
}

// In-place transpose of the 2^h x 2^h matrix at data (validated by callers).
bitrev_status_t run_transpose(void* data, int h, size_t s, hipStream_t st) {
  if (h == 0) return BITREV_SUCCESS;
  DeviceInfo d;
  bitrev_status_t status = device_info(&d, false);
  if (status != BITREV_SUCCESS) return status;
  const DefaultPlan dp = default_plan(0, (int)s, ((uint64_t)s) << (2 * h));
  int b = dp.b;
  if (b > h) b = h;
  if (b > max_tile_bits((int)s)) b = max_tile_bits((int)s);
  while (b > 0 && tile_lds_bytes_for((int)s, b, 2) > d.lds_per_block) --b;
  const size_t vb = (s << b) < 16 ? (s << b) : 16;
  TransposeLaunch a;
  a.data = data;
  a.h = h;
  const uint64_t nt = 1ull << (h - b);
  a.total_items = nt * (nt + 1) / 2;
  a.xcds = dp.xcd_remap == 2 ? 1 : d.xcds;
  a.grid = default_grid(a.total_items, d);
  const hipError_t e = launch_transpose((int)s, b, pointer_align(data, data) % vb == 0, a, st);
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

hipError_t launch_digit(int s, int d, int b, bool vec, const TileLaunch& a, hipStream_t st) {
  switch (s) {
    case 1: return launch_digit_s1(d, b, vec, a, st);
    case 2: return launch_digit_s2(d, b, vec, a, st);
    case 4: return launch_digit_s4(d, b, vec, a, st);
    case 8: return launch_digit_s8(d, b, vec, a, st);
    default: return launch_digit_s16(d, b, vec, a, st);
  }
}

hipError_t launch_wave_digit(int s, const WaveLaunch& a, int d, hipStream_t st) {
  switch (s) {
    case 1: return launch_wave_digit_s1(a, d, st);
    case 2: return launch_wave_digit_s2(a, d, st);
    case 4: return launch_wave_digit_s4(a, d, st);
    case 8: return launch_wave_digit_s8(a, d, st);
    default: return launch_wave_digit_s16(a, d, st);
  }
}

// Digit-reversed permutation (d-bit digits) of one array; src == dst in place.
// cfg (may be NULL): tile_bits (a whole number of digits), grid_blocks,
// order (out of place: the source tile order; in place the grouped digit
// order is fixed), xcd_remap and cache_hints as for the plain calls.
bitrev_status_t run_digit(const void* src, void* dst, int k, int d, size_t s,
                          const bitrev_config_t* cfg, void* stream) {
  // ---- validation: no HIP call before this block completes ----
  if (src == NULL || dst == NULL || k < 0 || k > BITREV_MAX_LOG2N || !valid_elem_size(s) ||
      d < 1 || d > 3 || k % d || !valid_config(cfg))
    return BITREV_ERROR_INVALID_VALUE;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % s)
    return BITREV_ERROR_INVALID_VALUE;
  const uint64_t n = 1ull << k;
  const bool inplace = (src == dst);
  if (!inplace && overlap(src, dst, (size_t)(n * s))) return BITREV_ERROR_ALIAS;
  if (d == 1) return run_plain(src, dst, k, 1, s, cfg, stream);
  if (inplace && k <= d) return BITREV_SUCCESS;  // one digit: the identity
  // ---- plan and launch ----
  DeviceInfo dev;
  bitrev_status_t st = device_info(&dev, false);
  if (st != BITREV_SUCCESS) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (k <= 6) {
    WaveLaunch w;
    w.src = src;
    w.dst = dst;
    w.k = k;
    w.nseg = 1;
    w.grid = 1;
    e = launch_wave_digit((int)s, w, d, hs);
    return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
  }
  const DefaultPlan dp = default_plan(inplace ? 0 : 1, (int)s, n * s);
  int b = dp.b;
  if (cfg && cfg->tile_bits) {
    b = cfg->tile_bits;  // forced: whole digits, within the array, compiled, fits
    if (b % d || 2 * b > k || b > max_tile_bits((int)s) ||
        tile_lds_bytes_for((int)s, b, 2) > dev.lds_per_block)
      return BITREV_ERROR_NOT_SUPPORTED;
  } else {
    // b must be a multiple of d: round up where the element size and the
    // array allow (radix 8 out of place, complex64 2^24: b = 3 moved 2.2 TB/s)
    const int bu = (b + d - 1) / d * d;
    if (bu <= max_tile_bits((int)s) && 2 * bu <= k) b = bu;
    if (b > max_tile_bits((int)s)) b = max_tile_bits((int)s);
    if (2 * b > k) b = k / 2;
    b -= b % d;
    while (b >= d && tile_lds_bytes_for((int)s, b, 2) > dev.lds_per_block) b -= d;
  }
  if (b < d) return BITREV_ERROR_NOT_SUPPORTED;
  const int m = k - 2 * b;
  if (m > 32) return BITREV_ERROR_NOT_SUPPORTED;
  TileLaunch a;
  a.src = src;
  a.dst = dst;
  a.m = m;
  a.total_items = inplace ? dpair_count(m, d) : (1ull << m);
  a.items_per_seg = a.total_items;
  a.seg_elems = n;
  // complex64 out of place at b = 6 measured otherwise at 2^24 (eight
  // alternating rounds): streaming loads rather than write-through stores,
  // and for radix 4 the grouped tile order in dispatch order (radix 4
  // 5236 -> 5547 GB/s, radix 8 5670 -> 5760)
  const bool c64_oop6 = !inplace && s == 8 && b == 6;
  a.balanced = (cfg && cfg->order) ? order_code(cfg->order) : ((c64_oop6 && d == 2) ? order_code(3) : 0);
  const int xr = (cfg && cfg->xcd_remap) ? cfg->xcd_remap : ((c64_oop6 && d == 2) ? 2 : dp.xcd_remap);
  a.xcds = xr == 2 ? 1 : dev.xcds;
  a.grid = (cfg && cfg->grid_blocks > 0) ? round_up((uint64_t)cfg->grid_blocks, (uint32_t)dev.xcds)
                                         : default_grid(a.total_items, dev);
  a.hints = (cfg && cfg->cache_hints)
                ? cfg->cache_hints - 1
                : default_hints(inplace ? kModeInplace : kModeOutofplace, (int)s, n * s, 1);
  if (!(cfg && cfg->cache_hints) && c64_oop6 && a.hints == kHintStreamWriteThrough)
    a.hints = kHintStreamLoads;
  a.pipelined = 0;
  const size_t vb = (s << b) < 16 ? (s << b) : 16;
  e = launch_digit((int)s, d, b, pointer_align(src, dst) % vb == 0, a, hs);
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

}  // namespace

extern "C" {

bitrev_status_t bitrev_digitrev_inplace(void* data, int log2n, int digit_bits, size_t elem_size,
                                        void* stream) {
  return run_digit(data, data, log2n, digit_bits, elem_size, NULL, stream);
}

bitrev_status_t bitrev_digitrev_outofplace(const void* src, void* dst, int log2n, int digit_bits,
                                           size_t elem_size, void* stream) {
  if (src != NULL && src == dst) return BITREV_ERROR_ALIAS;
  return run_digit(src, dst, log2n, digit_bits, elem_size, NULL, stream);
}

bitrev_status_t bitrev_digitrev_inplace_ex(void* data, int log2n, int digit_bits,
                                           size_t elem_size, const bitrev_config_t* cfg,
                                           void* stream) {
  return run_digit(data, data, log2n, digit_bits, elem_size, cfg, stream);
}

bitrev_status_t bitrev_digitrev_outofplace_ex(const void* src, void* dst, int log2n,
                                              int digit_bits, size_t elem_size,
                                              const bitrev_config_t* cfg, void* stream) {
  if (src != NULL && src == dst) return BITREV_ERROR_ALIAS;
  return run_digit(src, dst, log2n, digit_bits, elem_size, cfg, stream);
}

uint32_t bitrev_debug_digit_rev(uint32_t v, int j, int d) {
  return (j < 0 || j > 32 || d < 1 || d > 3) ? 0u : drev_bits(v, j, d);
}

uint64_t bitrev_debug_digit_pair_count(int m, int d) {
  return (m < 0 || m > 32 || d < 1 || d > 3 || m % d) ? 0 : dpair_count(m, d);
}

uint32_t bitrev_debug_digit_pair_at(int m, uint64_t w, int d) {
  if (m < 0 || m > 32 || d < 1 || d > 3 || m % d || w >= dpair_count(m, d)) return 0xFFFFFFFFu;
  return dpair_at(m, w, d);
}

uint32_t bitrev_debug_digit_inplace_pair_at(int m, uint64_t w, int d) {
  if (m < 0 || m > 32 || d < 1 || d > 3 || m % d || w >= dpair_count(m, d)) return 0xFFFFFFFFu;
  return dinplace_pair_at(m, w, d);
}

bitrev_status_t bitrev_transpose_inplace(void* data, int log2side, size_t elem_size, void* stream) {
  if (data == NULL || log2side < 0 || 2 * log2side > BITREV_MAX_LOG2N || !valid_elem_size(elem_size) ||
      reinterpret_cast<uintptr_t>(data) % elem_size)
    return BITREV_ERROR_INVALID_VALUE;
  if (log2side > 32) return BITREV_ERROR_NOT_SUPPORTED;
  return run_transpose(data, log2side, elem_size, static_cast<hipStream_t>(stream));
}

bitrev_status_t bitrev_dit_stages_ex(const void* src, void* dst, int log2n, int64_t rows,
                                     int stages, int inverse, int dtype,
                                     const bitrev_config_t* cfg, void* stream) {
  // ---- validation: no HIP call before this block completes ----
  if (src == NULL || dst == NULL || log2n < 0 || log2n > BITREV_MAX_LOG2N || rows < 0 ||
      stages < 0 || stages > 7 || (inverse != 0 && inverse != 1) || (dtype != 0 && dtype != 1) ||
      !valid_config(cfg))
    return BITREV_ERROR_INVALID_VALUE;
  const size_t s = dtype == 0 ? 8 : 16;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % s)
    return BITREV_ERROR_INVALID_VALUE;
  const uint64_t n = 1ull << log2n;
  if (rows > 0 && (uint64_t)rows > (1ull << 62) / (n * s)) return BITREV_ERROR_INVALID_VALUE;
  const bool inplace = (src == dst);
  if (!inplace && overlap(src, dst, (size_t)(n * s * (uint64_t)rows))) return BITREV_ERROR_ALIAS;
  if (2 * stages > log2n || stages > max_tile_bits((int)s)) return BITREV_ERROR_NOT_SUPPORTED;
  if (stages == 0) return run_plain(src, dst, log2n, rows, s, cfg, stream);
  if (rows == 0) return BITREV_SUCCESS;
  // ---- plan and launch ----
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  const DefaultPlan dp = default_plan(inplace ? 0 : 1, (int)s, n * s);
  int b;
  if (cfg && cfg->tile_bits) {
    b = cfg->tile_bits;  // forced: must hold the levels and fit
    if (2 * b > log2n || b > max_tile_bits((int)s)) return BITREV_ERROR_NOT_SUPPORTED;
  } else {
    // in place, complex64 takes b = 5 where the levels fit: the LDS passes
    // over a pair of 2^6-row tiles held two workgroups per CU
    // (complex64 2^24, 3-5 levels: 4864-5159 -> 5565-5717 GB/s)
    b = (inplace && s == 8) ? 5 : dp.b;
    if (b < stages) b = stages;
    if (b > max_tile_bits((int)s)) b = max_tile_bits((int)s);
    if (2 * b > log2n) b = log2n / 2;
  }
  const size_t lds = tile_lds_bytes_for((int)s, b, 2) + ((size_t)1 << b) * (s / 2);
  if (b < stages || lds > d.lds_per_block) return BITREV_ERROR_NOT_SUPPORTED;
  const int m = log2n - 2 * b;
  if (m > 32) return BITREV_ERROR_NOT_SUPPORTED;
  DitLaunch a;
  a.t.src = src;
  a.t.dst = dst;
  a.t.m = m;
  a.t.items_per_seg = inplace ? pair_count(m) : (1ull << m);
  a.t.total_items = a.t.items_per_seg * (uint64_t)rows;
  a.t.seg_elems = n;
  // grouped pairs in place, balanced tiles out of place; the XCD mapping and
  // cache hints of the plain kernel for this size.  Complex64 measured
  // otherwise (alternating rounds at 2^24-2^26): in place at b = 5 the
  // natural order up to 128 MiB (1-5 levels at 2^24 +3.4-3.9%; grouped is
  // 5-6% ahead at 256-512 MiB), with the write-through stores the hint table
  // gives it; in place at b = 6
  // streaming loads (best or tied at every size); out of place at b = 6 the
  // grouped order in dispatch order (+1.5% at 2^24)
  const uint64_t footprint = n * s * (uint64_t)rows;
  const bool c64_ip5 = inplace && s == 8 && b == 5;
  const bool c64_ip6 = inplace && s == 8 && b == 6;
  const bool c64_oop6 = !inplace && s == 8 && b == 6;
  const bool natural_ip5 = c64_ip5 && footprint <= (128ull << 20);
  a.t.balanced = order_code((cfg && cfg->order) ? cfg->order
                                                : (natural_ip5 ? 1 : ((inplace || c64_oop6) ? 3 : 2)));
  const int xr = (cfg && cfg->xcd_remap) ? cfg->xcd_remap : (c64_oop6 ? 2 : dp.xcd_remap);
  a.t.xcds = xr == 2 ? 1 : d.xcds;
  a.t.grid = (cfg && cfg->grid_blocks > 0) ? round_up((uint64_t)cfg->grid_blocks, (uint32_t)d.xcds)
                                           : default_grid(a.t.total_items, d);
  a.t.pipelined = 0;
  a.t.hints = (cfg && cfg->cache_hints)
                  ? cfg->cache_hints - 1
                  : default_hints(inplace ? kModeInplace : kModeOutofplace, (int)s, n * s, rows);
  if (!(cfg && cfg->cache_hints) && c64_ip6 && a.t.hints != kHintPlain)
    a.t.hints = kHintStreamLoads;
  a.stages = stages;
  a.inverse = inverse;
  const size_t vb = (s << b) < 16 ? (s << b) : 16;
  const bool vec = pointer_align(src, dst) % vb == 0;
  const hipError_t e = s == 8 ? launch_dit_s8(b, vec, a, static_cast<hipStream_t>(stream))
                              : launch_dit_s16(b, vec, a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

bitrev_status_t bitrev_dit_stages(const void* src, void* dst, int log2n, int64_t rows, int stages,
                                  int inverse, int dtype, void* stream) {
  return bitrev_dit_stages_ex(src, dst, log2n, rows, stages, inverse, dtype, NULL, stream);
}

// The block-local reversals with the second recursion level in LDS: 2^h
// contiguous blocks of 2^h elements each.
static bitrev_status_t run_block_recursive(void* data, int h, size_t s, hipStream_t st) {
  DeviceInfo d;
  bitrev_status_t status = device_info(&d, false);
  if (status != BITREV_SUCCESS) return status;
  const uint64_t nblocks = 1ull << h;
  // two 64 KiB blocks fit a compute unit's LDS at once
  const uint64_t cap = (uint64_t)d.cus * 8;
  const uint32_t grid = (uint32_t)(nblocks < cap ? nblocks : cap);
  const bool vec = reinterpret_cast<uintptr_t>(data) % 16 == 0 && (s << h) % 16 == 0;
  hipError_t e;
  switch (s) {
    case 1: e = launch_block_recursive_s1(data, h, nblocks, vec, grid, st); break;
    case 2: e = launch_block_recursive_s2(data, h, nblocks, vec, grid, st); break;
    case 4: e = launch_block_recursive_s4(data, h, nblocks, vec, grid, st); break;
    case 8: e = launch_block_recursive_s8(data, h, nblocks, vec, grid, st); break;
    default: e = launch_block_recursive_s16(data, h, nblocks, vec, grid, st); break;
  }
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

// Largest block the LDS stage of the second recursion level holds.
constexpr size_t kRecursiveBlockBytes = 65536;

bitrev_status_t bitrev_inplace_recursive_ex(void* data, int log2n, size_t elem_size, int levels,
                                            void* stream) {
  if (data == NULL || log2n < 0 || log2n > BITREV_MAX_LOG2N || !valid_elem_size(elem_size) ||
      reinterpret_cast<uintptr_t>(data) % elem_size || levels < 0 || levels > 2)
    return BITREV_ERROR_INVALID_VALUE;
  if (log2n % 2) return BITREV_ERROR_NOT_SUPPORTED;
  const int h = log2n / 2;
  const bool two_fit = h % 2 == 0 && (elem_size << h) <= kRecursiveBlockBytes;
  if (levels == 2 && !two_fit) return BITREV_ERROR_NOT_SUPPORTED;
  if (log2n <= 1) return BITREV_SUCCESS;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int64_t rows = (int64_t)1 << h;
  const bool two = levels == 2 || (levels == 0 && two_fit);
  bitrev_status_t st = two ? run_block_recursive(data, h, elem_size, hs)
                           : run_plain(data, data, h, rows, elem_size, NULL, stream);
  if (st == BITREV_SUCCESS) st = run_transpose(data, h, elem_size, hs);
  if (st == BITREV_SUCCESS)
    st = two ? run_block_recursive(data, h, elem_size, hs)
             : run_plain(data, data, h, rows, elem_size, NULL, stream);
  return st;
}

bitrev_status_t bitrev_inplace_recursive(void* data, int log2n, size_t elem_size, void* stream) {
  return bitrev_inplace_recursive_ex(data, log2n, elem_size, 0, stream);
}

bitrev_status_t bitrev_inplace(void* data, int log2n, size_t elem_size, void* stream) {
  return run_plain(data, data, log2n, 1, elem_size, NULL, stream);
}

bitrev_status_t bitrev_inplace_ex(void* data, int log2n, size_t elem_size,
                                  const bitrev_config_t* cfg, void* stream) {
  return run_plain(data, data, log2n, 1, elem_size, cfg, stream);
}

bitrev_status_t bitrev_inplace_timed(void* data, int log2n, size_t elem_size,
                                     const bitrev_config_t* cfg, void* start_event,
                                     void* stop_event, void* stream) {
  if (start_event == NULL || stop_event == NULL) return BITREV_ERROR_INVALID_VALUE;
  return run_plain(data, data, log2n, 1, elem_size, cfg, stream, 0, 0, start_event, stop_event);
}

bitrev_status_t bitrev_outofplace_timed(const void* src, void* dst, int log2n, size_t elem_size,
                                        const bitrev_config_t* cfg, void* start_event,
                                        void* stop_event, void* stream) {
  if (start_event == NULL || stop_event == NULL) return BITREV_ERROR_INVALID_VALUE;
  return run_plain(src, dst, log2n, 1, elem_size, cfg, stream, 0, 0, start_event, stop_event);
}

bitrev_status_t bitrev_timing_event_create(void** event) {
  if (event == NULL) return BITREV_ERROR_INVALID_VALUE;
  *event = NULL;
  hipEvent_t ev = NULL;
  // no system-scope fence when the event is reached: the stop timestamp is
  // then not delayed by the writeback of the L2 that such a fence performs
  const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableSystemFence);
  if (e != hipSuccess) return hip_fail(e);
  *event = (void*)ev;
  return BITREV_SUCCESS;
}

bitrev_status_t bitrev_timing_event_destroy(void* event) {
  if (event == NULL) return BITREV_SUCCESS;
  const hipError_t e = hipEventDestroy((hipEvent_t)event);
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

bitrev_status_t bitrev_timing_elapsed_ms(void* start_event, void* stop_event, float* ms) {
  if (start_event == NULL || stop_event == NULL || ms == NULL) return BITREV_ERROR_INVALID_VALUE;
  hipError_t e = hipEventSynchronize((hipEvent_t)stop_event);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, (hipEvent_t)start_event, (hipEvent_t)stop_event);
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

bitrev_status_t bitrev_outofplace(const void* src, void* dst, int log2n, size_t elem_size,
                                  void* stream) {
  if (src != NULL && src == dst) return BITREV_ERROR_ALIAS;
  return run_plain(src, dst, log2n, 1, elem_size, NULL, stream);
}

bitrev_status_t bitrev_outofplace_ex(const void* src, void* dst, int log2n, size_t elem_size,
                                     const bitrev_config_t* cfg, void* stream) {
  if (src != NULL && src == dst) return BITREV_ERROR_ALIAS;
  return run_plain(src, dst, log2n, 1, elem_size, cfg, stream);
}

bitrev_status_t bitrev_rows(const void* src, void* dst, int log2n, int64_t rows,
                            size_t elem_size, void* stream) {
  return run_plain(src, dst, log2n, rows, elem_size, NULL, stream);
}

bitrev_status_t bitrev_rows_ex(const void* src, void* dst, int log2n, int64_t rows,
                               size_t elem_size, const bitrev_config_t* cfg, void* stream) {
  return run_plain(src, dst, log2n, rows, elem_size, cfg, stream);
}

bitrev_status_t bitrev_rows_strided(const void* src, void* dst, int log2n, int64_t rows,
                                    int64_t src_stride, int64_t dst_stride, size_t elem_size,
                                    void* stream) {
  if (src_stride <= 0 || dst_stride <= 0) return BITREV_ERROR_INVALID_VALUE;
  return run_plain(src, dst, log2n, rows, elem_size, NULL, stream, (uint64_t)src_stride,
                   (uint64_t)dst_stride);
}

bitrev_status_t bitrev_evenodd(const void* src, void* dst, int log2n, int64_t rows,
                               size_t elem_size, void* stream) {
  if (src == NULL || dst == NULL || log2n < 1 || log2n > BITREV_MAX_LOG2N || rows < 0 ||
      !valid_elem_size(elem_size) ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % elem_size)
    return BITREV_ERROR_INVALID_VALUE;
  const uint64_t n = 1ull << log2n;
  if (rows > 0 && (uint64_t)rows > (1ull << 62) / (n * elem_size)) return BITREV_ERROR_INVALID_VALUE;
  const uint64_t bytes = n * elem_size * (uint64_t)rows;
  if (ranges_overlap(src, bytes, dst, bytes)) return BITREV_ERROR_ALIAS;
  if (rows == 0) return BITREV_SUCCESS;
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  const uint64_t pairs = (n / 2) * (uint64_t)rows;
  const uint64_t want = (pairs + 255) / 256;
  const uint32_t grid = (uint32_t)(want < (uint64_t)d.cus * 16 ? (want ? want : 1) : (uint64_t)d.cus * 16);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e;
  switch (elem_size) {
    case 1: e = launch_evenodd_s1(src, dst, log2n, (uint64_t)rows, grid, hs); break;
    case 2: e = launch_evenodd_s2(src, dst, log2n, (uint64_t)rows, grid, hs); break;
    case 4: e = launch_evenodd_s4(src, dst, log2n, (uint64_t)rows, grid, hs); break;
    case 8: e = launch_evenodd_s8(src, dst, log2n, (uint64_t)rows, grid, hs); break;
    default: e = launch_evenodd_s16(src, dst, log2n, (uint64_t)rows, grid, hs); break;
  }
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

size_t bitrev_batched_workspace_size(int64_t num_arrays) {
  if (num_arrays < 0 || num_arrays > (1ll << 40)) return 0;
  const size_t raw = ((size_t)num_arrays + 3) * 8;
  return (raw + 255) / 256 * 256;
}

// Common body of the batched entry points; src != NULL means out of place
// (src -> data, the same packed layout).
// Host-side checks of a batched call's arguments other than the workspace
// (no HIP call is made).  *nothing_to_do is set for num_arrays == 0.
static bitrev_status_t check_batched_args(const void* src, void* data, int64_t data_elems,
                                          const int64_t* offsets, const int32_t* log2n,
                                          int64_t num_arrays, size_t elem_size,
                                          const bitrev_config_t* cfg, bool* nothing_to_do) {
  *nothing_to_do = false;
  if (num_arrays < 0 || num_arrays > (1ll << 40) || data_elems < 0 || !valid_elem_size(elem_size) ||
      !valid_config(cfg))
    return BITREV_ERROR_INVALID_VALUE;
  if (num_arrays == 0) {
    *nothing_to_do = true;
    return BITREV_SUCCESS;
  }
  if (data == NULL || offsets == NULL || log2n == NULL) return BITREV_ERROR_INVALID_VALUE;
  if (reinterpret_cast<uintptr_t>(data) % elem_size || reinterpret_cast<uintptr_t>(offsets) % 8 ||
      reinterpret_cast<uintptr_t>(log2n) % 4)
    return BITREV_ERROR_INVALID_VALUE;
  if (src != NULL) {
    if (reinterpret_cast<uintptr_t>(src) % elem_size) return BITREV_ERROR_INVALID_VALUE;
    if ((uint64_t)data_elems > (1ull << 62) / elem_size) return BITREV_ERROR_INVALID_VALUE;
    const uint64_t bytes = (uint64_t)data_elems * elem_size;
    if (src == data || ranges_overlap(src, bytes, data, bytes)) return BITREV_ERROR_ALIAS;
  }
  return BITREV_SUCCESS;
}

static bitrev_status_t run_batched(const void* src, void* data, int64_t data_elems,
                                   const int64_t* offsets, const int32_t* log2n,
                                   int64_t num_arrays, size_t elem_size, void* workspace,
                                   size_t workspace_bytes, const bitrev_config_t* cfg,
                                   void* stream) {
  // ---- validation: no HIP call before this block completes ----
  bool nothing = false;
  const bitrev_status_t chk = check_batched_args(src, data, data_elems, offsets, log2n, num_arrays,
                                                 elem_size, cfg, &nothing);
  if (chk != BITREV_SUCCESS || nothing) return chk;
  if (workspace == NULL || reinterpret_cast<uintptr_t>(workspace) % 8 ||
      workspace_bytes < bitrev_batched_workspace_size(num_arrays))
    return BITREV_ERROR_WORKSPACE;
  // ---- plan and launch ----
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  Plan p;
  st = plan_batched((int)elem_size, cfg, d, true, src != NULL, &p);
  if (st != BITREV_SUCCESS) return st;
  BatchedLaunch a;
  a.src = src;
  a.data = data;
  a.offsets = offsets;
  a.log2n = log2n;
  a.num = num_arrays;
  a.data_elems = data_elems;
  a.ws = static_cast<int64_t*>(workspace);
  a.b = p.b;
  a.balanced = order_code(p.order);
  a.xcds = p.xcd_remap == 2 ? 1 : d.xcds;
  a.grid = p.grid;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = launch_batched_prep(a, hs);
  if (e != hipSuccess) return hip_fail(e);
  switch (elem_size) {
    case 1: e = launch_batched_s1(a, hs); break;
    case 2: e = launch_batched_s2(a, hs); break;
    case 4: e = launch_batched_s4(a, hs); break;
    case 8: e = launch_batched_s8(a, hs); break;
    default: e = launch_batched_s16(a, hs); break;
  }
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

bitrev_status_t bitrev_batched_ex(void* data, int64_t data_elems, const int64_t* offsets,
                                  const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                                  void* workspace, size_t workspace_bytes,
                                  const bitrev_config_t* cfg, void* stream) {
  return run_batched(NULL, data, data_elems, offsets, log2n, num_arrays, elem_size, workspace,
                     workspace_bytes, cfg, stream);
}

bitrev_status_t bitrev_batched_outofplace(const void* src, void* dst, int64_t data_elems,
                                          const int64_t* offsets, const int32_t* log2n,
                                          int64_t num_arrays, size_t elem_size, void* workspace,
                                          size_t workspace_bytes, void* stream) {
  if (src == NULL) return BITREV_ERROR_INVALID_VALUE;
  return run_batched(src, dst, data_elems, offsets, log2n, num_arrays, elem_size, workspace,
                     workspace_bytes, NULL, stream);
}

bitrev_status_t bitrev_batched(void* data, int64_t data_elems, const int64_t* offsets,
                               const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                               void* workspace, size_t workspace_bytes, void* stream) {
  return bitrev_batched_ex(data, data_elems, offsets, log2n, num_arrays, elem_size, workspace,
                           workspace_bytes, NULL, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free batched call: the workspace lives in a file-scope device
// array.  Host code never uses the array's name as an address (on the host it
// is only a stand-in for the symbol); it asks the runtime for the array's
// device address once per device and passes that to the kernels.
// ---------------------------------------------------------------------------
}  // extern "C"

// bitrev_batched_workspace_size(BITREV_NOALLOC_MAX_ARRAYS) bytes: the
// header and scan words, rounded up to 256 bytes
static __device__ __align__(256) int64_t scratch[(BITREV_NOALLOC_MAX_ARRAYS + 3 + 31) / 32 * 32];
static_assert(sizeof(scratch) == ((size_t)(BITREV_NOALLOC_MAX_ARRAYS + 3) * 8 + 255) / 256 * 256,
              "scratch must hold the workspace of the largest allowed batch");

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// The current device's address of `scratch`, looked up on the first call on
// each device with that device current.
bitrev_status_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= kMaxDevices) return hip_fail(hipErrorInvalidDevice);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BITREV_SUCCESS;
}
}  // namespace

extern "C" {

bitrev_status_t bitrev_batched_noalloc(void* data, int64_t data_elems, const int64_t* offsets,
                                       const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                                       void* stream) {
  // every argument, and the size limit, is checked before any HIP call
  bool nothing = false;
  const bitrev_status_t chk = check_batched_args(NULL, data, data_elems, offsets, log2n,
                                                 num_arrays, elem_size, NULL, &nothing);
  if (chk != BITREV_SUCCESS || nothing) return chk;
  if (num_arrays > BITREV_NOALLOC_MAX_ARRAYS) return BITREV_ERROR_WORKSPACE;
  void* ws = nullptr;
  const bitrev_status_t st = scratch_address(&ws);
  if (st != BITREV_SUCCESS) return st;
  // the prep kernel writes every workspace word the persistent kernel reads
  // (header and scan), so the previous call's contents need no clearing
  return run_batched(NULL, data, data_elems, offsets, log2n, num_arrays, elem_size, ws,
                     sizeof(scratch), NULL, stream);
}

bitrev_status_t bitrev_batched_errors(const void* workspace, int64_t* num_rejected,
                                      int64_t* first_rejected, void* stream) {
  if (workspace == NULL || reinterpret_cast<uintptr_t>(workspace) % 8) return BITREV_ERROR_WORKSPACE;
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  int64_t hdr[2] = {0, -1};
  e = hipMemcpy(hdr, workspace, sizeof hdr, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  if (num_rejected) *num_rejected = hdr[0];
  if (first_rejected) *first_rejected = hdr[1];
  return BITREV_SUCCESS;
}

bitrev_status_t bitrev_plan_query(int log2n, size_t elem_size, int64_t rows, int mode,
                                  const bitrev_config_t* cfg, bitrev_plan_t* plan) {
  if (plan == NULL || mode < 0 || mode > 2 || !valid_elem_size(elem_size) || !valid_config(cfg) ||
      rows < 0 || (mode != 2 && (log2n < 0 || log2n > BITREV_MAX_LOG2N)))
    return BITREV_ERROR_INVALID_VALUE;
  DeviceInfo d;
  bool have_device = false;
  bitrev_status_t st = device_info(&d, true, &have_device);
  if (st != BITREV_SUCCESS) return st;
  Plan p;
  st = (mode == 2) ? plan_batched((int)elem_size, cfg, d, have_device, false, &p)
                   : plan_plain(mode, log2n, (int)elem_size, rows, cfg, 16, d, have_device, &p);
  if (st != BITREV_SUCCESS) return st;
  memset(plan, 0, sizeof *plan);
  plan->path = p.path;
  plan->tile_bits = p.b;
  plan->mid_bits = p.m;
  plan->block_threads = p.threads;
  plan->grid_blocks = (int)p.grid;
  plan->order = p.order;
  plan->vector_access = p.vec ? 1 : 0;
  plan->variant = p.path == BITREV_PATH_TILE ? p.variant : 0;
  plan->xcd_remap = (p.path == BITREV_PATH_TILE || p.path == BITREV_PATH_BATCHED) ? p.xcd_remap : 0;
  plan->cache_hints = p.path == BITREV_PATH_TILE ? p.hints + 1 : 0;
  plan->work_items = p.total;
  plan->lds_bytes = p.lds;
  return BITREV_SUCCESS;
}

bitrev_status_t bitrev_load_tuning(const char* path) {
  load_env_tuning();  // an explicit load always wins over the environment
  return load_tuning_file(path);
}

const char* bitrev_tuning_format(void) { return kTuningFormat; }

bitrev_status_t bitrev_copy_ex(const void* src, void* dst, size_t bytes, int cache_hints,
                               void* stream) {
  if (src == NULL || dst == NULL || cache_hints < 0 || cache_hints > 4)
    return BITREV_ERROR_INVALID_VALUE;
  if (bytes == 0) return BITREV_SUCCESS;
  if (overlap(src, dst, bytes)) return BITREV_ERROR_ALIAS;
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  // streaming loads with write-through stores: the fastest form measured at
  // 128 MiB and at 4 GiB (plain and streaming-load copies trail by 1-4%)
  const int h = cache_hints ? cache_hints - 1 : kHintStreamWriteThrough;
  const hipError_t e = launch_copy(src, dst, bytes, (uint32_t)(d.cus * 4), h,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

bitrev_status_t bitrev_copy(const void* src, void* dst, size_t bytes, void* stream) {
  return bitrev_copy_ex(src, dst, bytes, 0, stream);
}

bitrev_status_t bitrev_copy_tiled(const void* src, void* dst, int log2n, size_t elem_size,
                                  const bitrev_config_t* cfg, void* stream) {
  // ---- validation: no HIP call before this block completes ----
  if (src == NULL || dst == NULL || log2n < 0 || log2n > BITREV_MAX_LOG2N ||
      !valid_elem_size(elem_size) || !valid_config(cfg) ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % elem_size)
    return BITREV_ERROR_INVALID_VALUE;
  const uint64_t bytes = (uint64_t)elem_size << log2n;
  if (overlap(src, dst, (size_t)bytes)) return BITREV_ERROR_ALIAS;
  // ---- plan and launch ----
  DeviceInfo d;
  bitrev_status_t st = device_info(&d, false);
  if (st != BITREV_SUCCESS) return st;
  Plan p;
  st = plan_plain(kModeOutofplace, log2n, (int)elem_size, 1, cfg, pointer_align(src, dst), d, true,
                  &p);
  if (st != BITREV_SUCCESS) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (p.path != BITREV_PATH_TILE) {
    // arrays of at most 64 elements have no tiles: a plain copy
    const hipError_t e = launch_copy(src, dst, (size_t)bytes, 1, kHintPlain, hs);
    return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
  }
  if (!p.vec) return BITREV_ERROR_NOT_SUPPORTED;
  TileLaunch a;
  a.src = src;
  a.dst = dst;
  a.m = p.m;
  a.items_per_seg = a.total_items = 1ull << p.m;
  a.seg_elems = a.dst_seg_elems = 1ull << log2n;
  a.balanced = order_code(p.order);
  a.xcds = p.xcd_remap == 2 ? 1 : d.xcds;
  a.grid = (cfg && cfg->grid_blocks > 0) ? p.grid : default_grid(a.total_items, d);
  a.pipelined = 0;
  a.hints = p.hints;
  hipError_t e;
  switch (elem_size) {
    case 1: e = launch_tile_copy_s1(p.b, a, hs); break;
    case 2: e = launch_tile_copy_s2(p.b, a, hs); break;
    case 4: e = launch_tile_copy_s4(p.b, a, hs); break;
    case 8: e = launch_tile_copy_s8(p.b, a, hs); break;
    default: e = launch_tile_copy_s16(p.b, a, hs); break;
  }
  return e == hipSuccess ? BITREV_SUCCESS : hip_fail(e);
}

const char* bitrev_status_string(bitrev_status_t status) {
  switch (status) {
    case BITREV_SUCCESS: return "success";
    case BITREV_ERROR_INVALID_VALUE: return "invalid value";
    case BITREV_ERROR_ALIAS: return "source and destination overlap";
    case BITREV_ERROR_WORKSPACE: return "workspace missing, misaligned or too small";
    case BITREV_ERROR_HIP: return "HIP runtime error";
    case BITREV_ERROR_NOT_SUPPORTED: return "not supported by this build or device";
  }
  return "unknown status";
}

int bitrev_last_hip_error(void) { return g_last_hip_error; }

int bitrev_abi_version(void) { return BITREV_ABI_VERSION; }

uint32_t bitrev_debug_rev(uint32_t v, int j) {
  return (j < 0 || j > 32) ? 0u : rev_bits(v, j);
}

uint64_t bitrev_debug_pair_count(int m) { return (m < 0 || m > 32) ? 0 : pair_count(m); }

uint32_t bitrev_debug_pair_at(int m, uint64_t w, int balanced) {
  if (m < 0 || m > 32 || w >= pair_count(m)) return 0xFFFFFFFFu;
  return pair_at(m, w, balanced != 0);
}

uint32_t bitrev_debug_oop_tile_at(int m, uint32_t w, int order) {
  if (m < 0 || m > 32 || (m < 32 && w >= (1u << m)) || order < 1 || order > 3) return 0xFFFFFFFFu;
  return oop_tile_at(m, w, order_code(order));
}

uint32_t bitrev_debug_inplace_pair_at(int m, uint64_t w, int order) {
  if (m < 0 || m > 32 || w >= pair_count(m) || order < 1 || order > 3) return 0xFFFFFFFFu;
  return inplace_pair_at(m, w, order_code(order));
}

void bitrev_debug_tri_pair(uint64_t w, uint32_t* r, uint32_t* c) {
  uint32_t rr = 0, cc = 0;
  tri_pair(w, &rr, &cc);
  if (r) *r = rr;
  if (c) *c = cc;
}

uint32_t bitrev_debug_spread(uint32_t w, int width) {
  return (width < 0 || width > 32) ? 0u : spread_bits(w, width);
}

}  // extern "C"
