// Batched form of the method: many frame pairs of different sizes with the same levels,
// radius and iteration count.  Every (level, iteration) phase is one launch whose
// workgroups stride over a work list of tiles of all pairs; the pyramid steps are batched
// the same way.  The whole schedule of a batch is captured once per set of caller buffers
// into a hipGraph and replayed.  Tile height and workgroup count per level come from a
// configuration the autotuner can search.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ofmi.h"
#include "kernels.h"
#include "runtime.h"

using namespace ofmi;

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


struct LevelCfg {
  int nb;     // tile height in bands of 2R+1 rows
  int grid;   // iteration workgroups; 0 = one per tile
  int variant;   // TileVariant, or -1: by tile count
};

// Argument blocks of a batch: one per cached graph (OF_BATCH_GRAPHS pointer sets) and a ring
// of OF_BATCH_EAGER_SLOTS for eager runs.
constexpr int kGraphSlots = OF_BATCH_GRAPHS;
constexpr int kEagerSlots = OF_BATCH_EAGER_SLOTS;
constexpr int kArgSlots = kGraphSlots + kEagerSlots;

}  // namespace

struct of_batch {
  int n = 0, L = 0, R = 0, K = 0;
  unsigned flags = 0;
  int device = 0;
  std::vector<Geometry> g;          // per pair
  std::vector<size_t> pair_off;     // workspace offset of each pair's buffers
  char* ws = nullptr;               // workspace (pair buffers, work lists, eager arguments)
  bool owns_ws = false;
  size_t off_tiles = 0, cap_tiles = 0;   // int4 tile lists of all levels (capacity per level)
  size_t off_items = 0;                  // int2 pyramid items of all levels
  size_t off_args = 0;                   // eager argument block
  size_t arg_bytes = 0;
  std::vector<int> ntiles, nitems;
  std::vector<int> nactive;         // per level: tiles with an unmasked pixel, first in the list
  std::vector<char> partial;        // per level: a listed tile holds masked pixels
  std::vector<size_t> items_at;
  LevelCfg cfg[OF_MAX_LEVELS];
  // Argument slots (arg_bytes each, device slots in the workspace from off_args, pinned host
  // copies in `pinned`): kGraphSlots for captured graphs, then kEagerSlots as a ring for eager
  // runs.  slot_done[i] is recorded after the last launch that reads slot i.
  char* pinned = nullptr;
  char* pinned_dev = nullptr;   // the pinned slots' device mapping (read by the copy kernel)
  hipEvent_t slot_done[kArgSlots] = {};
  bool slot_used[kArgSlots] = {};
  int eager_next = 0;
  std::vector<std::pair<std::vector<uintptr_t>, int>> graph_slot;   // pointer set -> slot
  // Masks (of_batch_set_masks): per masked pair, its mask pyramid in `maskbuf` (offsets per
  // level) and a host copy from which the work lists take their tile flags and row cuts.  A
  // masked pair also gets four flow planes of its own per level >= 1 in `maskbuf`
  // (plane_off), so that no level writes over another's zero regions: the zero regions of
  // every intermediate plane are cleared once per tile configuration and only the final
  // phase visits the tiles without an unmasked pixel.
  uint8_t* maskbuf = nullptr;
  std::vector<std::vector<size_t>> mask_off;      // [pair][level]
  std::vector<std::vector<size_t>> plane_off;     // [pair][level >= 1] u0, u1, v0, v1 planes
  std::vector<std::vector<std::vector<uint8_t>>> hmask;   // [pair][level] host copies
  KernelTimer timer;
  GraphCache graphs;
};

namespace {

of_status hip_fail(const char* what, hipError_t e) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return OF_EHIP;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

// Bytes of the argument block: pyramid jobs of all reduce steps, then the iteration
// arguments of all phases.
size_t args_bytes(int n, int L, int K) {
  return align256(sizeof(ReduceJob) * 2 * (size_t)n * (L > 1 ? L - 1 : 0)) +
         align256(sizeof(IterArgs) * (size_t)n * L * (K > 0 ? K : 1));
}

bool check_batch(int n, const int* H, const int* W, int levels, int radius, int iters,
                 unsigned flags) {
  if (n < 1 || n > 65536) return set_error("batch size out of range"), false;
  if (flags & OF_FLAG_NORMALIZE) return set_error("OF_FLAG_NORMALIZE applies to plans only"), false;
  if (flags & OF_FLAG_GRAPH) return set_error("OF_FLAG_GRAPH applies to plans only"), false;
  if (!H || !W) return set_error("NULL size arrays"), false;
  for (int i = 0; i < n; ++i)
    if (!check_params(H[i], W[i], levels, radius, iters, flags)) {
      set_error("pair " + std::to_string(i) + ": " + of_last_error());
      return false;
    }
  return true;
}

int default_batch_bands(const of_batch* b, int l) {
  long long px = 0;
  for (int i = 0; i < b->n; ++i) px += (long long)b->g[i].H[l] * b->g[i].W[l];
  // Many pairs fill the device even with tall tiles, which cut the vertical halo.
  if (px >= (24ll << 20)) return 4;
  if (px >= (4ll << 20)) return 2;
  return 1;
}

// Work items one pair's level can need at any tile height: the one-band tiles, or at taller
// tiles every tile plus up to two zero items per tile cut to its unmasked bands (a two-band
// tile loses at most one end, a taller one both: at most two more items per tile column than
// the one-band tiles).
size_t list_capacity(int H, int W, int N, int TW) {
  return (size_t)((W + TW - 1) / TW) * ((H + N - 1) / N + 2);
}

// Tile flags of masked pair p at level l for the current tile height (0: no unmasked pixel,
// 1: some, 2: all); empty for an unmasked pair.
std::vector<uint8_t> pair_flags(const of_batch* b, int p, int l) {
  if (!b->maskbuf || b->mask_off[p].empty()) return {};
  const Geometry& g = b->g[p];
  return tile_flags(b->hmask[p][l].data(), g.H[l], g.W[l], strip_width_for(b->R),
                    (2 * b->R + 1) * b->cfg[l].nb);
}

// Tile work lists of all levels for the current configuration (work items: pair | tile flag
// << 16, tile x, first row, rows).  Each tile's height is cut to the bands the frame holds
// (a tile at the bottom edge would otherwise run all its configured bands), and a tile with
// masked pixels to its bands that hold unmasked rows (the masked rows cut off go to the zero
// list).  The tiles with an unmasked pixel come first
// (nactive of them), the all-masked ones after them.  For masked pairs every intermediate
// flow plane is cleared: the phases before the final one write only the listed active tiles,
// so the rest stays zero.  Set-up calls only: no run may be in flight.
hipError_t upload_tiles(of_batch* b) {
  const int TW = strip_width_for(b->R), N = 2 * b->R + 1;
  for (int l = 0; l < b->L; ++l) {
    const int TH = N * b->cfg[l].nb;
    std::vector<int4> act, off;
    b->partial[l] = 0;
    for (int p = 0; p < b->n; ++p) {
      const int H = b->g[p].H[l], W = b->g[p].W[l];
      const std::vector<uint8_t> f = pair_flags(b, p, l);
      const int tx = (W + TW - 1) / TW, ty = (H + TH - 1) / TH;
      for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x) {
          const int fl = f.empty() ? 2 : f[(size_t)y * tx + x];
          const int y0 = y * TH, e = std::min(H, y0 + TH);
          if (fl == 0) {
            off.push_back(make_int4(p, x, y0, e - y0));
            continue;
          }
          int ty0 = y0, th = std::min(TH, (e - y0 + N - 1) / N * N);
          if (fl == 1) {
            // from the first to the last band with an unmasked row; bands stay where the
            // tile's bands are (multiples of 2r+1 from row 0), since the window sums combine
            // per-band partial sums and so round by where the band boundaries fall
            b->partial[l] = 1;
            band_cut(b->hmask[p][l].data(), W, x * TW, std::min(W, x * TW + TW), y0, e, N, ty0, th);
            if (ty0 > y0) off.push_back(make_int4(p, x, y0, ty0 - y0));
            if (ty0 + th < e) off.push_back(make_int4(p, x, ty0 + th, e - (ty0 + th)));
          }
          act.push_back(make_int4(p | (fl << 16), x, ty0, th));
        }
    }
    b->nactive[l] = (int)act.size();
    act.insert(act.end(), off.begin(), off.end());
    if (act.size() > b->cap_tiles) return hipErrorInvalidValue;
    b->ntiles[l] = (int)act.size();
    hipError_t e = hipMemcpy(b->ws + b->off_tiles + l * b->cap_tiles * sizeof(int4), act.data(),
                             act.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipSuccess;
  for (int p = 0; p < b->n && e == hipSuccess && b->maskbuf; ++p) {
    if (b->mask_off[p].empty()) continue;
    const Geometry& g = b->g[p];
    const size_t n0 = (size_t)g.H[0] * g.W[0] * sizeof(float);
    for (int i = 0; i < 4 && e == hipSuccess; ++i)
      e = hipMemset(b->ws + b->pair_off[p] + g.off_flow[i], 0, n0);
    for (int l = 1; l < b->L && e == hipSuccess; ++l)
      e = hipMemset(b->maskbuf + b->plane_off[p][l], 0,
                    4 * (size_t)g.H[l] * g.W[l] * sizeof(float));
  }
  return e;
}

// Fill the argument block for the given caller buffers.
void fill_args(const of_batch* b, char* blk, const void* const* I1, const void* const* I2,
               float* const* u, float* const* v) {
  const int n = b->n, L = b->L, K = b->K;
  ReduceJob* jobs = (ReduceJob*)blk;
  IterArgs* args =
      (IterArgs*)(blk + align256(sizeof(ReduceJob) * 2 * (size_t)n * (L > 1 ? L - 1 : 0)));
  for (int p = 0; p < n; ++p) {
    const Geometry& g = b->g[p];
    char* ws = b->ws + b->pair_off[p];
    const void* P1[OF_MAX_LEVELS];
    const void* P2[OF_MAX_LEVELS];
    P1[0] = I1[p];
    P2[0] = I2[p];
    for (int l = 1; l < L; ++l) {
      P1[l] = ws + g.off_p1[l];
      P2[l] = ws + g.off_p2[l];
      ReduceJob* j = jobs + (size_t)(l - 1) * 2 * n + 2 * p;
      j[0] = {P1[l - 1], (void*)P1[l], g.H[l - 1], g.W[l - 1], g.H[l], g.W[l]};
      j[1] = {P2[l - 1], (void*)P2[l], g.H[l - 1], g.W[l - 1], g.H[l], g.W[l]};
    }
    const bool masked = b->maskbuf && !b->mask_off[p].empty();
    const float* cu = nullptr;
    const float* cv = nullptr;
    int cH = 0, cW = 0, buf = 0, phase = 0;
    for (int l = L - 1; l >= 0; --l) {
      float* fu[2] = {(float*)(ws + g.off_flow[0]), (float*)(ws + g.off_flow[1])};
      float* fv[2] = {(float*)(ws + g.off_flow[2]), (float*)(ws + g.off_flow[3])};
      if (masked && l > 0) {
        float* pl = (float*)(b->maskbuf + b->plane_off[p][l]);
        const size_t nl = (size_t)g.H[l] * g.W[l];
        fu[0] = pl;
        fu[1] = pl + nl;
        fv[0] = pl + 2 * nl;
        fv[1] = pl + 3 * nl;
      }
      for (int k = 0; k < K; ++k, ++phase) {
        IterArgs& a = args[(size_t)phase * n + p];
        a = IterArgs{};
        a.I1 = P1[l];
        a.I2 = P2[l];
        a.H = g.H[l];
        a.W = g.W[l];
        a.uin = cu;
        a.vin = cv;
        a.Hc = cH;
        a.Wc = cW;
        a.mode = k > 0 ? kFlowSame : (l == L - 1 ? kFlowZero : kFlowCoarse);
        const bool last = (l == 0 && k == K - 1);
        a.uout = last ? u[p] : fu[buf];
        a.vout = last ? v[p] : fv[buf];
        if (b->flags & OF_FLAG_GAUSSIAN_WINDOW) gaussian_taps(a.taps, b->R);
        if (masked) a.mask = b->maskbuf + b->mask_off[p][l];
        cu = a.uout;
        cv = a.vout;
        cH = a.H;
        cW = a.W;
        buf ^= 1;
      }
    }
  }
}

// Enqueue the whole schedule reading arguments from device block `blk`.
hipError_t enqueue_batch(of_batch* b, char* blk, float* const* u, float* const* v,
                         hipStream_t s, KernelTimer* t) {
  const int n = b->n, L = b->L, K = b->K;
  if (K == 0) {
    for (int p = 0; p < n; ++p) {
      hipError_t e = launch_zero(u[p], v[p], (size_t)b->g[p].H[0] * b->g[p].W[0], s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const Geometry& g0 = b->g[0];
  const ReduceJob* jobs = (const ReduceJob*)blk;
  const IterArgs* args =
      (const IterArgs*)(blk + align256(sizeof(ReduceJob) * 2 * (size_t)n * (L > 1 ? L - 1 : 0)));
  hipEvent_t span = nullptr;
  double span_units = 0, span_bytes = 0;
  if (t && t->per_level() && L > 1) {
    hipError_t e = t->begin(s, &span);
    if (e != hipSuccess) return e;
  }
  for (int l = 1; l < L; ++l) {
    hipEvent_t ev = nullptr;
    hipError_t e = t && t->per_launch() ? t->begin(s, &ev) : hipSuccess;
    const int ni = b->nitems[l];
    if (e == hipSuccess)
      e = launch_reduce_batch(g0.elem(l - 1), g0.ep, jobs + (size_t)(l - 1) * 2 * n,
                              (const int2*)(b->ws + b->items_at[l]), ni, std::min(ni, 8192), s);
    if (e == hipSuccess && t) {
      double no = 0, bytes = 0;
      for (int p = 0; p < n; ++p) {
        const double o = (double)b->g[p].H[l] * b->g[p].W[l];
        const double i = (double)b->g[p].H[l - 1] * b->g[p].W[l - 1];
        no += 2 * o;
        bytes += 2 * (i * elem_bytes(g0.elem(l - 1)) + o * elem_bytes(g0.ep));
      }
      if (t->per_launch()) e = t->end(s, ev, OF_KERNEL_REDUCE, no, bytes);
      span_units += no;
      span_bytes += bytes;
    }
    if (e != hipSuccess) return e;
  }
  if (span) {
    hipError_t e = t->end(s, span, OF_KERNEL_REDUCE, span_units, span_bytes, L - 1);
    if (e != hipSuccess) return e;
  }
  int phase = 0;
  for (int l = L - 1; l >= 0; --l) {
    double px = 0;
    for (int p = 0; p < n; ++p) px += (double)b->g[p].H[l] * b->g[p].W[l];
    hipEvent_t lspan = nullptr;
    if (t && t->per_level()) {
      hipError_t e = t->begin(s, &lspan);
      if (e != hipSuccess) return e;
    }
    for (int k = 0; k < K; ++k, ++phase) {
      BatchLaunch bl;
      bl.args = args + (size_t)phase * n;
      bl.tiles = (const int4*)(b->ws + b->off_tiles + l * b->cap_tiles * sizeof(int4));
      // Every phase computes the tiles with an unmasked pixel only.  The all-masked tiles
      // after them in the list hold zeros in the intermediate planes from set-up; the final
      // phase zero-fills them in the caller's planes with a launch of their own (inside the
      // iteration launch, the contiguous per-XCD ranges of the list would leave some XCDs
      // only zero tiles).
      bl.ntiles = b->nactive[l];
      const int nzero = (l == 0 && k == K - 1) ? b->ntiles[l] - b->nactive[l] : 0;
      bl.grid = b->cfg[l].grid > 0 ? std::min(b->cfg[l].grid, bl.ntiles) : bl.ntiles;
      bl.grid = (bl.grid + 7) / 8 * 8;
      bl.variant = b->cfg[l].variant >= 0 ? b->cfg[l].variant : default_tile_variant(b->ntiles[l]);
      if (b->flags & OF_FLAG_GAUSSIAN_WINDOW) bl.variant |= kTileGauss;
      // Only tiles that hold masked and unmasked pixels need the masked kernel.
      bl.masked = b->maskbuf != nullptr && b->partial[l];
      const int mode = k > 0 ? kFlowSame : (l == L - 1 ? kFlowZero : kFlowCoarse);
      hipEvent_t ev = nullptr;
      hipError_t e = t && t->per_launch() ? t->begin(s, &ev) : hipSuccess;
      if (e == hipSuccess && bl.ntiles > 0) e = launch_iter_batch(g0.elem(l), bl, b->R, mode, s);
      if (e == hipSuccess && nzero > 0)
        e = launch_zero_tiles(bl.args, bl.tiles + bl.ntiles, nzero, strip_width_for(b->R), s);
      if (e == hipSuccess && t && t->per_launch())
        e = t->end(s, ev, OF_KERNEL_ITERATE, px, px * (2.0 * elem_bytes(g0.elem(l)) + 16.0));
      if (e != hipSuccess) return e;
    }
    if (lspan) {
      hipError_t e = t->end(s, lspan, OF_KERNEL_LEVEL(l), px * K,
                            px * K * (2.0 * elem_bytes(g0.elem(l)) + 16.0), K);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

char* dev_slot(const of_batch* b, int i) { return b->ws + b->off_args + (size_t)i * b->arg_bytes; }
char* host_slot(const of_batch* b, int i) { return b->pinned + (size_t)i * b->arg_bytes; }
// A slot's arguments reach the device through a copy kernel that reads the pinned slot through
// its device mapping (the runtime's asynchronous host-to-device copy from pinned memory was seen
// to block the calling thread for milliseconds now and then).
hipError_t upload_slot(const of_batch* b, int i, hipStream_t s) {
  return launch_copy(dev_slot(b, i), b->pinned_dev + (size_t)i * b->arg_bytes, b->arg_bytes, s);
}

// Is slot i free for new arguments (no launch in flight reads it)?  hipErrorNotReady if busy.
hipError_t slot_free(of_batch* b, int i) {
  if (!b->slot_used[i]) return hipSuccess;
  return hipEventQuery(b->slot_done[i]);
}

// Eager path: the arguments go through the next pinned slot of the eager ring into its device
// slot; a slot still read by an earlier run makes the call return busy (hipErrorNotReady).
hipError_t run_eager(of_batch* b, const void* const* I1, const void* const* I2, float* const* u,
                     float* const* v, hipStream_t s, KernelTimer* t) {
  const int slot = kGraphSlots + b->eager_next;
  hipError_t e = slot_free(b, slot);
  if (e != hipSuccess) return e;
  fill_args(b, host_slot(b, slot), I1, I2, u, v);
  e = upload_slot(b, slot, s);
  if (e == hipSuccess) e = enqueue_batch(b, dev_slot(b, slot), u, v, s, t);
  if (e == hipSuccess) e = hipEventRecord(b->slot_done[slot], s);
  if (e != hipSuccess) return e;
  b->slot_used[slot] = true;
  b->eager_next = (b->eager_next + 1) % kEagerSlots;
  return hipSuccess;
}

void drop_graphs(of_batch* b) {
  hipDeviceSynchronize();
  b->graphs.clear();
  b->graph_slot.clear();
}

}  // namespace

extern "C" {

size_t of_batch_workspace_bytes(int n, const int* H, const int* W, int levels, int radius,
                                int iters, unsigned flags) {
  if (!check_batch(n, H, W, levels, radius, iters, flags)) return 0;
  size_t off = 0, tiles = 0, items = 0;
  const int N = 2 * radius + 1, TW = strip_width_for(radius);
  for (int l = 0; l < levels; ++l) {
    size_t tl = 0, it = 0;
    for (int p = 0; p < n; ++p) {
      Geometry g = make_geometry(H[p], W[p], levels, radius, iters, flags);
      if (l == 0) off += align256(g.bytes);
      tl += list_capacity(g.H[l], g.W[l], N, TW);
      if (l >= 1) it += 2 * (size_t)reduce_blocks(g.H[l], g.W[l]);
    }
    tiles = std::max(tiles, tl);
    items += align256(it * sizeof(int2));
  }
  return off + align256(tiles * sizeof(int4)) * levels + items + kArgSlots * args_bytes(n, levels, iters);
}

of_batch* of_batch_create(int n, const int* H, const int* W, int levels, int radius, int iters,
                          unsigned flags, void* workspace, size_t workspace_bytes) {
  if (!check_batch(n, H, W, levels, radius, iters, flags)) return nullptr;
  const size_t need = of_batch_workspace_bytes(n, H, W, levels, radius, iters, flags);
  if (workspace && workspace_bytes < need) {
    set_error("workspace smaller than of_batch_workspace_bytes()");
    return nullptr;
  }
  if (workspace && ((uintptr_t)workspace & 255)) {
    set_error("workspace must be 256-byte aligned");
    return nullptr;
  }
  of_batch* b = new of_batch();
  b->n = n;
  b->L = levels;
  b->R = radius;
  b->K = iters;
  b->flags = flags;
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    hip_fail("hipGetDevice", e);
    delete b;
    return nullptr;
  }
  size_t off = 0;
  for (int p = 0; p < n; ++p) {
    b->g.push_back(make_geometry(H[p], W[p], levels, radius, iters, flags));
    b->pair_off.push_back(off);
    off += align256(b->g.back().bytes);
  }
  const int N = 2 * radius + 1, TW = strip_width_for(radius);
  size_t cap = 0;
  for (int l = 0; l < levels; ++l) {
    size_t tl = 0;
    for (int p = 0; p < n; ++p) tl += list_capacity(b->g[p].H[l], b->g[p].W[l], N, TW);
    cap = std::max(cap, tl);
  }
  b->cap_tiles = align256(cap * sizeof(int4)) / sizeof(int4);
  b->off_tiles = off;
  off += b->cap_tiles * sizeof(int4) * levels;
  b->off_items = off;
  b->ntiles.assign(levels, 0);
  b->nactive.assign(levels, 0);
  b->partial.assign(levels, 0);
  b->nitems.assign(levels, 0);
  b->items_at.assign(levels, 0);
  std::vector<std::vector<int2>> items(levels);
  for (int l = 1; l < levels; ++l) {
    for (int p = 0; p < n; ++p) {
      const int blocks = reduce_blocks(b->g[p].H[l], b->g[p].W[l]);
      for (int f = 0; f < 2; ++f)
        for (int k = 0; k < blocks; ++k) items[l].push_back(make_int2(2 * p + f, k));
    }
    b->items_at[l] = off;
    b->nitems[l] = (int)items[l].size();
    off += align256(items[l].size() * sizeof(int2));
  }
  b->off_args = off;
  b->arg_bytes = args_bytes(n, levels, iters);
  off += kArgSlots * b->arg_bytes;
  if (off != need) {
    set_error("internal: workspace layout mismatch");
    delete b;
    return nullptr;
  }
  if (workspace) {
    b->ws = (char*)workspace;
  } else {
    e = hipMalloc((void**)&b->ws, need);
    if (e != hipSuccess) {
      hip_fail("hipMalloc(batch workspace)", e);
      delete b;
      return nullptr;
    }
    b->owns_ws = true;
  }
  for (int l = 0; l < levels; ++l) b->cfg[l] = {default_batch_bands(b, l), 0, -1};
  e = upload_tiles(b);
  for (int l = 1; l < levels && e == hipSuccess; ++l)
    e = hipMemcpy(b->ws + b->items_at[l], items[l].data(), items[l].size() * sizeof(int2),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->pinned, kArgSlots * b->arg_bytes, hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&b->pinned_dev, b->pinned, 0);
  for (int i = 0; i < kArgSlots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&b->slot_done[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    hip_fail("batch set-up", e);
    of_batch_destroy(b);
    return nullptr;
  }
  return b;
}

of_status of_batch_compute(of_batch* b, const void* const* I1, const void* const* I2,
                           float* const* u, float* const* v, void* stream) {
  if (!b) return set_error("NULL batch"), OF_EINVAL;
  if (!I1 || !I2 || !u || !v) return set_error("NULL pointer array"), OF_EINVAL;
  for (int p = 0; p < b->n; ++p) {
    if (!I1[p] || !I2[p] || !u[p] || !v[p])
      return set_error("NULL buffer of pair " + std::to_string(p)), OF_EINVAL;
    if (u[p] == v[p] || (((uintptr_t)u[p] | (uintptr_t)v[p]) & 3))
      return set_error("bad output planes of pair " + std::to_string(p)), OF_EINVAL;
  }
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (b->timer.on || (b->flags & OF_FLAG_NO_GRAPH)) {
    e = run_eager(b, I1, I2, u, v, s, &b->timer);
  } else {
    std::vector<uintptr_t> key;
    key.reserve(4 * (size_t)b->n);
    for (int p = 0; p < b->n; ++p) {
      key.push_back((uintptr_t)I1[p]);
      key.push_back((uintptr_t)I2[p]);
      key.push_back((uintptr_t)u[p]);
      key.push_back((uintptr_t)v[p]);
    }
    int slot = -1;
    for (const auto& gs : b->graph_slot)
      if (gs.first == key) slot = gs.second;
    const bool fresh = slot < 0;
    e = hipSuccess;
    if (fresh) {
      // A new pointer set: a free graph slot, else the least recently used graph's slot once
      // its last replay has completed (the only wait of this call).
      bool taken[kGraphSlots] = {};
      for (const auto& gs : b->graph_slot) taken[gs.second] = true;
      for (int i = 0; i < kGraphSlots && slot < 0; ++i)
        if (!taken[i]) slot = i;
      if (slot < 0 && b->graphs.entries.empty()) {   // only after failed captures
        b->graph_slot.clear();
        slot = 0;
        e = hipEventSynchronize(b->slot_done[slot]);
      }
      if (slot < 0) {
        const size_t lru = b->graphs.lru();
        const std::vector<uintptr_t> old = b->graphs.entries[lru].key;
        for (size_t i = 0; i < b->graph_slot.size(); ++i)
          if (b->graph_slot[i].first == old) {
            slot = b->graph_slot[i].second;
            b->graph_slot.erase(b->graph_slot.begin() + i);
            break;
          }
        e = hipEventSynchronize(b->slot_done[slot]);
        if (e == hipSuccess) b->graphs.erase(lru);
      }
      if (e == hipSuccess) {
        fill_args(b, host_slot(b, slot), I1, I2, u, v);
        e = upload_slot(b, slot, s);
      }
    }
    char* blk = dev_slot(b, slot);
    if (e == hipSuccess)
      e = b->graphs.run(key, s, [&](hipStream_t cs) { return enqueue_batch(b, blk, u, v, cs, nullptr); });
    if (e == hipSuccess && fresh) b->graph_slot.push_back({key, slot});
    if (e == hipSuccess) e = hipEventRecord(b->slot_done[slot], s);
    if (e == hipSuccess) b->slot_used[slot] = true;
  }
  if (e == hipErrorNotReady)
    return set_error("busy: every eager argument slot is read by a run still in flight"), OF_ESTATE;
  if (e != hipSuccess) return hip_fail("batch launch", e), OF_EHIP;
  return OF_OK;
}

void of_batch_destroy(of_batch* b) {
  if (!b) return;
  DeviceGuard guard(b->device);
  hipDeviceSynchronize();
  drop_graphs(b);
  for (int i = 0; i < kArgSlots; ++i)
    if (b->slot_done[i]) hipEventDestroy(b->slot_done[i]);
  if (b->pinned) hipHostFree(b->pinned);
  if (b->maskbuf) hipFree(b->maskbuf);
  if (b->owns_ws) hipFree(b->ws);
  delete b;
}

of_status of_batch_set_masks(of_batch* b, const uint8_t* const* masks, void* stream) {
  if (!b) return set_error("NULL batch"), OF_EINVAL;
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipDeviceSynchronize();   // captured graphs and runs in flight hold the old masks
  if (e != hipSuccess) return hip_fail("set_masks", e);
  drop_graphs(b);
  if (b->maskbuf) hipFree(b->maskbuf);
  b->maskbuf = nullptr;
  b->mask_off.assign(b->n, {});
  b->plane_off.assign(b->n, {});
  b->hmask.assign(b->n, {});
  bool any = false;
  for (int p = 0; masks && p < b->n; ++p) any |= masks[p] != nullptr;
  if (!any) {   // every tile active again
    e = upload_tiles(b);
    return e == hipSuccess ? OF_OK : hip_fail("set_masks", e);
  }
  // layout: mask pyramids and flow planes of levels >= 1 of the masked pairs
  size_t mtotal = 0;
  for (int p = 0; p < b->n; ++p) {
    if (!masks[p]) continue;
    const Geometry& g = b->g[p];
    for (int l = 0; l < b->L; ++l) {
      b->mask_off[p].push_back(mtotal);
      mtotal += align256((size_t)g.H[l] * g.W[l]);
    }
    b->plane_off[p].assign(b->L, 0);
    for (int l = 1; l < b->L; ++l) {
      b->plane_off[p][l] = mtotal;
      mtotal += align256(4 * (size_t)g.H[l] * g.W[l] * sizeof(float));
    }
  }
  e = hipMalloc((void**)&b->maskbuf, mtotal);
  for (int p = 0; p < b->n && e == hipSuccess; ++p) {
    if (!masks[p]) continue;
    const Geometry& g = b->g[p];
    e = hipMemcpyAsync(b->maskbuf + b->mask_off[p][0], masks[p], (size_t)g.H[0] * g.W[0],
                       hipMemcpyDeviceToDevice, s);
    for (int l = 1; l < b->L && e == hipSuccess; ++l)
      e = launch_mask_reduce(b->maskbuf + b->mask_off[p][l - 1], g.H[l - 1], g.W[l - 1],
                             b->maskbuf + b->mask_off[p][l], g.H[l], g.W[l], s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (int p = 0; p < b->n && e == hipSuccess; ++p) {
    if (!masks[p]) continue;
    b->hmask[p].resize(b->L);
    for (int l = 0; l < b->L && e == hipSuccess; ++l) {
      b->hmask[p][l].resize((size_t)b->g[p].H[l] * b->g[p].W[l]);
      e = hipMemcpy(b->hmask[p][l].data(), b->maskbuf + b->mask_off[p][l], b->hmask[p][l].size(),
                    hipMemcpyDeviceToHost);
    }
  }
  if (e == hipSuccess) e = upload_tiles(b);
  if (e != hipSuccess) {
    if (b->maskbuf) hipFree(b->maskbuf);
    b->maskbuf = nullptr;
    b->mask_off.assign(b->n, {});
    b->plane_off.assign(b->n, {});
    upload_tiles(b);
    return hip_fail("set_masks", e);
  }
  return OF_OK;
}

of_status of_batch_set_timing(of_batch* b, int enable) {
  if (!b) return set_error("NULL batch"), OF_EINVAL;
  if (enable < 0 || enable > OF_TIMING_LEVEL) return set_error("unknown timing mode"), OF_EINVAL;
  b->timer.on = enable != 0;
  if (enable) b->timer.mode = enable;
  return OF_OK;
}

of_status of_batch_read_timing(of_batch* b, int kernel, double* total_ms, long long* launches,
                               double* units, double* bytes) {
  if (!b) return set_error("NULL batch"), OF_EINVAL;
  if (kernel != OF_KERNEL_ITERATE && kernel != OF_KERNEL_REDUCE &&
      !(kernel >= OF_KERNEL_LEVEL(0) && kernel < OF_KERNEL_LEVEL(OF_MAX_LEVELS)))
    return set_error("unknown kernel id"), OF_EINVAL;
  DeviceGuard guard(b->device);
  hipError_t e = b->timer.read(kernel, total_ms, launches, units, bytes);
  if (e != hipSuccess) return hip_fail("timing events", e);
  return OF_OK;
}

of_status of_batch_get_config(const of_batch* b, int* bands, int* grid, int* variant) {
  if (!b || !bands || !grid) return set_error("NULL argument"), OF_EINVAL;
  for (int l = 0; l < b->L; ++l) {
    bands[l] = b->cfg[l].nb;
    grid[l] = b->cfg[l].grid;
    if (variant) variant[l] = b->cfg[l].variant;
  }
  return OF_OK;
}

of_status of_batch_set_config(of_batch* b, const int* bands, const int* grid, const int* variant) {
  if (!b || !bands || !grid) return set_error("NULL argument"), OF_EINVAL;
  for (int l = 0; l < b->L; ++l)
    if (bands[l] < 1 || bands[l] > 64 || grid[l] < 0 ||
        (variant && (variant[l] < -1 || variant[l] > kTileWideLean)))
      return set_error("config out of range"), OF_EINVAL;
  DeviceGuard guard(b->device);
  drop_graphs(b);
  for (int l = 0; l < b->L; ++l) b->cfg[l] = {bands[l], grid[l], variant ? variant[l] : -1};
  hipError_t e = upload_tiles(b);
  if (e != hipSuccess) return hip_fail("tile lists", e);
  return OF_OK;
}

of_status of_batch_autotune(of_batch* b, const void* const* I1, const void* const* I2,
                            float* const* u, float* const* v, void* stream, int reps) {
  if (!b || !I1 || !I2 || !u || !v) return set_error("NULL argument"), OF_EINVAL;
  if (reps < 1) reps = 1;
  DeviceGuard guard(b->device);
  hipStream_t s = (hipStream_t)stream;
  const bool was_on = b->timer.on;
  const int was_mode = b->timer.mode;
  b->timer.on = true;
  b->timer.mode = OF_TIMING_LAUNCH;
  static const int kBands[] = {1, 2, 4, 8, 16};
  static const int kGrid[] = {0, 256, 512, 1024, 2048};
  static const int kVariant[] = {kTileNarrow, kTileWide, kTileWideLean};
  hipError_t e = hipSuccess;
  // Coordinate descent, one level at a time: the iteration time of that level only.
  for (int l = 0; l < b->L && e == hipSuccess; ++l) {
    int maxH = 0;
    for (int p = 0; p < b->n; ++p) maxH = std::max(maxH, b->g[p].H[l]);
    double best = 1e30;
    LevelCfg bestc = b->cfg[l];
    for (int nb : kBands) {
      if (nb > 1 && (2 * b->R + 1) * nb > 2 * maxH) continue;
      for (int gr : kGrid)
      for (int wd : kVariant) {
        b->cfg[l] = {nb, gr, wd};
        e = upload_tiles(b);
        if (e != hipSuccess) break;
        double tl = 1e30;
        for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
          e = run_eager(b, I1, I2, u, v, s, &b->timer);
          if (e != hipSuccess) break;
          // Launch k of level l is the ((L-1-l)*K + k)-th iteration launch of the run.
          std::vector<KernelTimer::Rec> mine;
          e = hipStreamSynchronize(s);
          if (e != hipSuccess) break;
          int idx = 0;
          double sum = 0;
          const int first = (b->L - 1 - l) * b->K;
          for (const KernelTimer::Rec& rc : b->timer.recs) {
            if (rc.kernel != OF_KERNEL_ITERATE) continue;
            if (idx >= first && idx < first + b->K) {
              float ms = 0;
              hipEventElapsedTime(&ms, rc.a, rc.b);
              sum += ms;
            }
            ++idx;
          }
          double d1, d2, d3;
          long long n1;
          b->timer.read(OF_KERNEL_ITERATE, &d1, &n1, &d2, &d3);
          b->timer.read(OF_KERNEL_REDUCE, &d1, &n1, &d2, &d3);
          if (r > 0) tl = std::min(tl, sum);
        }
        if (e == hipSuccess && tl < best) {
          best = tl;
          bestc = {nb, gr, wd};
        }
      }
    }
    b->cfg[l] = bestc;
    if (e == hipSuccess) e = upload_tiles(b);
  }
  b->timer.on = was_on;
  b->timer.mode = was_mode;
  drop_graphs(b);
  if (e != hipSuccess) return hip_fail("autotune", e);
  return OF_OK;
}

}  // extern "C"
