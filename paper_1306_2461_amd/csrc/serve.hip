// Serving form: frame streams whose previous frame's pyramid stays resident on the device, so
// each new pair builds one new pyramid (the paper's first computing scheme, Sec. 2.4: each
// field needs only one new image processed).  A server admits streams against an HBM budget
// and pushes the new frames of many streams together: one batched launch per pyramid step
// and per (level, iteration) phase over the tiles of every stream in the push.
//
// A push's launch arguments (pyramid jobs, per-session iteration arguments, tile lists) are
// packed on the host into one of kRing pinned staging slots, copied to the matching device
// slot on the push's stream and read by the kernels there.  Slots are sized when a session
// opens, for a push of every open session, so a push never allocates; a slot is reused only
// once the event recorded after its push's last launch has completed, and a push that finds
// its slot still in flight returns OF_ESTATE instead of waiting.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ofmi.h"
#include "kernels.h"
#include "runtime.h"

using namespace ofmi;

namespace {

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

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

of_status hip_fail(const char* what, hipError_t e) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return OF_EHIP;
}

constexpr int kRing = OF_SERVER_RING;   // staging slots per server (pushes in flight at once)

}  // namespace

struct of_server;

struct of_session {
  of_server* server = nullptr;
  int H = 0, W = 0;
  Geometry g;                     // level sizes
  char* mem = nullptr;            // slots and flow planes
  bool owns_mem = false;          // allocated by the library (else caller workspace)
  size_t bytes = 0;
  size_t slot_off[2][OF_MAX_LEVELS];  // pyramid planes of the two frame slots
  char* flow = nullptr;           // four level-0 FP32 planes
  int cur = 0;                    // slot that receives the next frame
  bool has_prev = false;
  // mask (of_session_set_mask): mask pyramid and four FP32 flow planes per level >= 1 in one
  // allocation, so that no level writes over another's zero regions: every intermediate plane
  // holds zero at the masked pixels from set-up on (the launches write zero there too), so
  // the all-masked tiles are left out of all but the final phase.  The tile flags of every
  // push tile height, and the band cuts of the tiles with masked pixels (first row, rows), are
  // kept on the host, where the push work lists are built.
  uint8_t* maskbuf = nullptr;
  size_t mask_off[OF_MAX_LEVELS] = {};
  size_t flag_off[3][OF_MAX_LEVELS] = {};
  size_t plane_off[OF_MAX_LEVELS] = {};
  std::vector<uint8_t> hflags;
  std::vector<int2> hcut;
};

struct of_server {
  int L = 0, R = 0, K = 0;
  unsigned flags = 0;
  int device = 0;
  size_t budget = 0;
  size_t resident = 0;
  bool hidden = false;            // created for of_session_create (no budget)
  std::vector<of_session*> sessions;
  // staging ring: kRing device and pinned host slots of slot_bytes each
  char* dev_blk = nullptr;
  char* host_blk = nullptr;
  char* host_blk_dev = nullptr;   // the pinned slots' device mapping (read by the copy kernel)
  size_t slot_bytes = 0;
  hipEvent_t done[kRing] = {};
  bool in_use[kRing] = {};
  int next = 0;
  std::mutex mu;
};

namespace {

// Loads every iteration kernel a push of this server may launch (each level's frame type and
// field source, the wide and wide lean tiles, with or without masks) on the current device, so
// that no push pays a kernel's first-launch code load (about 10 ms measured on a request).
hipError_t prime_push_kernels(const of_server* s, bool masked) {
  const int side = 1 << (s->L - 1);
  const Geometry g = make_geometry(side, side, s->L, s->R, s->K, s->flags);
  BatchLaunch bl{};
  bl.prime = true;
  bl.masked = masked;
  for (int l = 0; l < s->L; ++l)
    for (int k = 0; k < std::min(s->K, 2); ++k)
      for (int v : {(int)kTileWide, (int)kTileWideLean}) {
        bl.variant = v | ((s->flags & OF_FLAG_GAUSSIAN_WINDOW) ? kTileGauss : 0);
        const int mode = k > 0 ? kFlowSame : (l == s->L - 1 ? kFlowZero : kFlowCoarse);
        const hipError_t e = launch_iter_batch(g.elem(l), bl, s->R, mode, nullptr);
        if (e != hipSuccess) return e;
      }
  return masked ? prime_zero_tiles() : hipSuccess;
}

size_t session_bytes(int H, int W, int L, int R, int K, unsigned flags, Geometry* gout,
                     size_t slot_off[2][OF_MAX_LEVELS], size_t* flow_off) {
  Geometry g = make_geometry(H, W, L, R, K, flags);
  size_t off = 0;
  for (int s = 0; s < 2; ++s)
    for (int l = 0; l < L; ++l) {
      if (slot_off) slot_off[s][l] = off;
      off += align256((size_t)g.H[l] * g.W[l] * elem_bytes(g.elem(l)));
    }
  if (flow_off) *flow_off = off;
  off += 4 * align256((size_t)H * W * sizeof(float));
  if (gout) *gout = g;
  return off;
}

// Host-side description of one push, packed into one staging slot.
struct Push {
  std::vector<std::vector<ReduceJob>> jobs;   // per output level 1..L-1
  std::vector<std::vector<int2>> items;
  std::vector<std::vector<IterArgs>> args;    // per phase, one per flowing session
  std::vector<std::vector<int4>> tiles;       // per level, over flowing sessions
  std::vector<int> nactive;                   // per level: tiles with an unmasked pixel, first
  std::vector<char> partial;                  // per level: a listed tile holds masked pixels
  size_t bytes = 0;
  std::vector<size_t> off_jobs, off_items, off_args, off_tiles;
};

void layout(Push& p) {
  size_t off = 0;
  auto put = [&](size_t n) {
    const size_t o = off;
    off += align256(n);
    return o;
  };
  for (auto& j : p.jobs) p.off_jobs.push_back(put(j.size() * sizeof(ReduceJob)));
  for (auto& i : p.items) p.off_items.push_back(put(i.size() * sizeof(int2)));
  for (auto& a : p.args) p.off_args.push_back(put(a.size() * sizeof(IterArgs)));
  for (auto& t : p.tiles) p.off_tiles.push_back(put(t.size() * sizeof(int4)));
  p.bytes = off;
}

void pack(const Push& p, char* dst) {
  for (size_t i = 0; i < p.jobs.size(); ++i)
    memcpy(dst + p.off_jobs[i], p.jobs[i].data(), p.jobs[i].size() * sizeof(ReduceJob));
  for (size_t i = 0; i < p.items.size(); ++i)
    memcpy(dst + p.off_items[i], p.items[i].data(), p.items[i].size() * sizeof(int2));
  for (size_t i = 0; i < p.args.size(); ++i)
    memcpy(dst + p.off_args[i], p.args[i].data(), p.args[i].size() * sizeof(IterArgs));
  for (size_t i = 0; i < p.tiles.size(); ++i)
    memcpy(dst + p.off_tiles[i], p.tiles[i].data(), p.tiles[i].size() * sizeof(int4));
}

// Tile height (bands) of a push level: taller tiles when many pixels fill the device.
int push_bands(long long px) { return px >= (24ll << 20) ? 4 : (px >= (4ll << 20) ? 2 : 1); }

// Upper bound of the staging bytes of a push of every session in `ss` (all flowing, one-band
// tiles, every array padded to 256 bytes): a push of any subset packs into fewer bytes.
size_t push_bound(const std::vector<of_session*>& ss, int L, int R, int K) {
  const int TW = strip_width_for(R), N = 2 * R + 1;
  const size_t n = ss.size();
  size_t b = 0;
  for (int l = 1; l < L; ++l) {
    size_t items = 0;
    for (const of_session* x : ss) items += reduce_blocks(x->g.H[l], x->g.W[l]);
    b += align256(n * sizeof(ReduceJob)) + align256(items * sizeof(int2));
  }
  b += (size_t)L * (K > 0 ? K : 0) * align256(n * sizeof(IterArgs));
  for (int l = 0; l < L; ++l) {
    size_t tiles = 0;
    // one-band tiles, or taller tiles plus up to two zero items per tile cut to its unmasked
    // bands: at most two more items per tile column
    for (const of_session* x : ss)
      tiles += (size_t)((x->g.W[l] + TW - 1) / TW) * ((x->g.H[l] + N - 1) / N + 2);
    b += align256(tiles * sizeof(int4));
  }
  return b;
}

void free_ring(of_server* s) {
  if (s->dev_blk) hipFree(s->dev_blk);
  if (s->host_blk) hipHostFree(s->host_blk);
  s->host_blk_dev = nullptr;
  s->dev_blk = nullptr;
  s->host_blk = nullptr;
  s->slot_bytes = 0;
  for (int i = 0; i < kRing; ++i) s->in_use[i] = false;
}

// Grows the staging ring to `need` bytes per slot (set-up calls only: waits for the device,
// since pushes in flight read the old slots).
hipError_t reserve_ring(of_server* s, size_t need) {
  if (need <= s->slot_bytes) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return e;
  free_ring(s);
  const size_t sb = align256(need + need / 4);
  e = hipMalloc((void**)&s->dev_blk, sb * kRing);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_blk, sb * kRing, hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&s->host_blk_dev, s->host_blk, 0);
  if (e != hipSuccess) {
    free_ring(s);
    return e;
  }
  s->slot_bytes = sb;
  return hipSuccess;
}

bool check_server_flags(unsigned flags) {
  if (flags & OF_FLAG_NORMALIZE) return set_error("OF_FLAG_NORMALIZE applies to plans only"), false;
  if (flags & OF_FLAG_GRAPH) return set_error("OF_FLAG_GRAPH applies to plans only"), false;
  return true;
}

// Tile heights (in bands) a push may choose (push_bands) and their slot in a session's flags.
constexpr int kPushBands[3] = {1, 2, 4};
int band_slot(int nb) { return nb == 1 ? 0 : (nb == 2 ? 1 : 2); }

// Servers behind of_session_create, one per (device, levels, radius, iters, flags).
std::mutex g_hidden_mu;
std::map<std::tuple<int, int, int, int, unsigned>, of_server*> g_hidden;

of_session* open_session(of_server* s, int H, int W, void* workspace, size_t workspace_bytes) {
  if (!check_params(H, W, s->L, s->R, s->K, s->flags)) return nullptr;
  std::lock_guard<std::mutex> lock(s->mu);
  of_session* ss = new of_session();
  size_t flow_off = 0;
  ss->bytes = session_bytes(H, W, s->L, s->R, s->K, s->flags, &ss->g, ss->slot_off, &flow_off);
  if (s->budget && s->resident + ss->bytes > s->budget) {
    set_error("HBM budget exceeded: stream needs " + std::to_string(ss->bytes) + " bytes, " +
              std::to_string(s->budget - s->resident) + " left");
    delete ss;
    return nullptr;
  }
  if (workspace) {
    if (workspace_bytes < ss->bytes) {
      set_error("workspace smaller than of_session_bytes()");
      delete ss;
      return nullptr;
    }
    if ((uintptr_t)workspace & 255) {
      set_error("workspace must be 256-byte aligned");
      delete ss;
      return nullptr;
    }
  }
  DeviceGuard guard(s->device);
  ss->server = s;
  ss->H = H;
  ss->W = W;
  std::vector<of_session*> all = s->sessions;
  all.push_back(ss);
  hipError_t e = reserve_ring(s, push_bound(all, s->L, s->R, s->K));
  if (e != hipSuccess) {
    hip_fail("staging ring", e);
    delete ss;
    return nullptr;
  }
  if (workspace) {
    ss->mem = (char*)workspace;
  } else {
    e = hipMalloc((void**)&ss->mem, ss->bytes);
    if (e != hipSuccess) {
      hip_fail("hipMalloc(session)", e);
      delete ss;
      return nullptr;
    }
    ss->owns_mem = true;
  }
  ss->flow = ss->mem + flow_off;
  s->resident += ss->bytes;
  s->sessions.push_back(ss);
  return ss;
}

void destroy_server(of_server* s) {
  DeviceGuard guard(s->device);
  hipDeviceSynchronize();
  for (of_session* ss : s->sessions) {
    if (ss->owns_mem) hipFree(ss->mem);
    if (ss->maskbuf) hipFree(ss->maskbuf);
    delete ss;
  }
  free_ring(s);
  for (int i = 0; i < kRing; ++i)
    if (s->done[i]) hipEventDestroy(s->done[i]);
  delete s;
}

}  // namespace

extern "C" {

size_t of_session_bytes(int H, int W, int levels, int radius, int iters, unsigned flags) {
  if (!check_params(H, W, levels, radius, iters, flags)) return 0;
  if (!check_server_flags(flags & ~OF_FLAG_NO_GRAPH)) return 0;
  return session_bytes(H, W, levels, radius, iters, flags, nullptr, nullptr, nullptr);
}

of_server* of_server_create(int levels, int radius, int iters, unsigned flags,
                            size_t hbm_budget_bytes) {
  flags &= ~OF_FLAG_NO_GRAPH;
  if (!check_server_flags(flags)) return nullptr;
  if (!check_params(1 << (levels > 0 ? levels - 1 : 0), 1 << (levels > 0 ? levels - 1 : 0), levels,
                    radius, iters, flags))
    return nullptr;
  of_server* s = new of_server();
  s->L = levels;
  s->R = radius;
  s->K = iters;
  s->flags = flags;
  s->budget = hbm_budget_bytes;
  hipError_t e = hipGetDevice(&s->device);
  for (int i = 0; i < kRing && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming);
  if (e == hipSuccess) e = prime_push_kernels(s, false);
  if (e != hipSuccess) {
    hip_fail("server set-up", e);
    destroy_server(s);
    return nullptr;
  }
  return s;
}

size_t of_server_resident_bytes(const of_server* s) { return s ? s->resident : 0; }

of_session* of_server_open(of_server* s, int H, int W) {
  if (!s) return set_error("NULL server"), nullptr;
  return open_session(s, H, W, nullptr, 0);
}

of_session* of_server_open_ex(of_server* s, int H, int W, void* workspace, size_t workspace_bytes) {
  if (!s) return set_error("NULL server"), nullptr;
  return open_session(s, H, W, workspace, workspace_bytes);
}

size_t of_session_resident_bytes(const of_session* ss) { return ss ? ss->bytes : 0; }

of_status of_server_close(of_server* s, of_session* ss) {
  if (!s || !ss || ss->server != s) return set_error("bad server or session"), OF_EINVAL;
  std::lock_guard<std::mutex> lock(s->mu);
  DeviceGuard guard(s->device);
  hipDeviceSynchronize();
  if (ss->owns_mem) hipFree(ss->mem);
  if (ss->maskbuf) hipFree(ss->maskbuf);
  s->resident -= ss->bytes;
  s->sessions.erase(std::remove(s->sessions.begin(), s->sessions.end(), ss), s->sessions.end());
  delete ss;
  return OF_OK;
}

of_status of_server_push(of_server* s, of_session* const* ss, int n, const void* const* frames,
                         float* const* u, float* const* v, int* has_flow, void* stream) {
  if (!s || !ss || !frames || !u || !v || !has_flow) return set_error("NULL argument"), OF_EINVAL;
  if (n < 1) return set_error("n must be >= 1"), OF_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ss[i] || ss[i]->server != s) return set_error("session of another server"), OF_EINVAL;
    if (!frames[i]) return set_error("NULL frame"), OF_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ss[j] == ss[i]) return set_error("a session appears twice in one push"), OF_EINVAL;
    if (ss[i]->has_prev && (!u[i] || !v[i] || u[i] == v[i] || (((uintptr_t)u[i] | (uintptr_t)v[i]) & 3)))
      return set_error("bad output planes"), OF_EINVAL;
  }
  std::lock_guard<std::mutex> lock(s->mu);
  DeviceGuard guard(s->device);
  hipStream_t st = (hipStream_t)stream;
  const int slot = s->next;
  if (s->in_use[slot]) {
    const hipError_t q = hipEventQuery(s->done[slot]);
    if (q == hipErrorNotReady)
      return set_error("busy: every staging slot is held by a push still in flight"), OF_ESTATE;
    if (q != hipSuccess) return hip_fail("staging slot", q);
  }
  const int L = s->L, K = s->K, R = s->R;
  const Geometry& gg = ss[0]->g;
  // 1. describe the push
  Push p;
  p.jobs.resize(L > 1 ? L - 1 : 0);
  p.items.resize(L > 1 ? L - 1 : 0);
  for (int l = 1; l < L; ++l)
    for (int i = 0; i < n; ++i) {
      of_session* x = ss[i];
      const int job = (int)p.jobs[l - 1].size();
      p.jobs[l - 1].push_back({x->mem + x->slot_off[x->cur][l - 1], x->mem + x->slot_off[x->cur][l],
                               x->g.H[l - 1], x->g.W[l - 1], x->g.H[l], x->g.W[l]});
      const int blocks = reduce_blocks(x->g.H[l], x->g.W[l]);
      for (int k = 0; k < blocks; ++k) p.items[l - 1].push_back(make_int2(job, k));
    }
  std::vector<int> flowing;
  for (int i = 0; i < n; ++i)
    if (ss[i]->has_prev && K > 0) flowing.push_back(i);
  if (flowing.size() > 65536)   // work items carry the session index in 16 bits
    return set_error("more than 65536 flowing sessions in one push"), OF_EINVAL;
  const int TW = strip_width_for(R), N = 2 * R + 1;
  p.args.resize((size_t)L * (K > 0 ? K : 0));
  p.tiles.resize(L);
  p.nactive.assign(L, 0);
  p.partial.assign(L, 0);
  int level_bands[OF_MAX_LEVELS];
  for (int l = L - 1; l >= 0; --l) {
    long long px = 0;
    for (int i : flowing) px += (long long)ss[i]->g.H[l] * ss[i]->g.W[l];
    level_bands[l] = push_bands(px);
    const int TH = N * level_bands[l];
    std::vector<int4> off;   // all-masked tiles, after the active ones
    for (int q = 0; q < (int)flowing.size(); ++q) {
      const of_session* x = ss[flowing[q]];
      const size_t fo = x->maskbuf ? x->flag_off[band_slot(level_bands[l])][l] : 0;
      const uint8_t* f = x->maskbuf ? x->hflags.data() + fo : nullptr;
      const int tx = (x->g.W[l] + TW - 1) / TW, ty = (x->g.H[l] + TH - 1) / TH;
      for (int yy = 0; yy < ty; ++yy)
        for (int xx = 0; xx < tx; ++xx) {
          const int fl = f ? f[(size_t)yy * tx + xx] : 2;
          p.partial[l] |= fl == 1;
          // work item (session | flag << 16, tile x, first row, rows): the height cut to the
          // bands the frame holds, a tile with masked pixels to its bands with unmasked rows
          // (the rows cut off are zero-filled in the final phase)
          const int y0 = yy * TH, e = std::min(x->g.H[l], y0 + TH);
          if (fl == 0) {
            off.push_back(make_int4(q, xx, y0, e - y0));
            continue;
          }
          int ty0 = y0, th = (e - y0 + N - 1) / N * N;
          if (fl == 1) {
            const int2 c = x->hcut[fo + (size_t)yy * tx + xx];
            ty0 = c.x;
            th = c.y;
            if (ty0 > y0) off.push_back(make_int4(q, xx, y0, ty0 - y0));
            if (ty0 + th < e) off.push_back(make_int4(q, xx, ty0 + th, e - (ty0 + th)));
          }
          p.tiles[l].push_back(make_int4(q | (fl << 16), xx, ty0, th));
        }
    }
    p.nactive[l] = (int)p.tiles[l].size();
    p.tiles[l].insert(p.tiles[l].end(), off.begin(), off.end());
  }
  for (int q = 0; q < (int)flowing.size(); ++q) {
    const int i = flowing[q];
    of_session* x = ss[i];
    const int prev = x->cur ^ 1;
    const size_t fb = align256((size_t)x->H * x->W * 4);
    const float* cu = nullptr;
    const float* cv = nullptr;
    int cH = 0, cW = 0, buf = 0, phase = 0;
    for (int l = L - 1; l >= 0; --l) {
      float* fu[2] = {(float*)(x->flow), (float*)(x->flow + fb)};
      float* fv[2] = {(float*)(x->flow + 2 * fb), (float*)(x->flow + 3 * fb)};
      if (x->maskbuf && l > 0) {
        float* pl = (float*)(x->maskbuf + x->plane_off[l]);
        const size_t nl = (size_t)x->g.H[l] * x->g.W[l];
        fu[0] = pl;
        fu[1] = pl + nl;
        fv[0] = pl + 2 * nl;
        fv[1] = pl + 3 * nl;
      }
      for (int k = 0; k < K; ++k, ++phase) {
        IterArgs a{};
        a.I1 = x->mem + x->slot_off[prev][l];
        a.I2 = x->mem + x->slot_off[x->cur][l];
        a.H = x->g.H[l];
        a.W = x->g.W[l];
        a.uin = cu;
        a.vin = cv;
        a.Hc = cH;
        a.Wc = cW;
        a.mode = k > 0 ? kFlowSame : (l == L - 1 ? kFlowZero : kFlowCoarse);
        const bool last = (l == 0 && k == K - 1);
        a.uout = last ? u[i] : fu[buf];
        a.vout = last ? v[i] : fv[buf];
        if (s->flags & OF_FLAG_GAUSSIAN_WINDOW) gaussian_taps(a.taps, R);
        if (x->maskbuf) a.mask = x->maskbuf + x->mask_off[l];
        p.args[phase].push_back(a);
        cu = a.uout;
        cv = a.vout;
        cH = a.H;
        cW = a.W;
        buf ^= 1;
      }
    }
  }
  layout(p);
  if (p.bytes > s->slot_bytes)   // cannot happen for sessions opened on this server
    return set_error("internal: push larger than the staging slots"), OF_ESTATE;
  char* hblk = s->host_blk + (size_t)slot * s->slot_bytes;
  char* dblk = s->dev_blk + (size_t)slot * s->slot_bytes;
  pack(p, hblk);
  // 2. new frames into their slots (level 0), the arguments into the device slot.  Both are
  // copy kernels on the push's stream (the arguments read from the pinned slot through its
  // device mapping): the runtime's asynchronous host-to-device copy from pinned memory blocked
  // the calling thread for about 9 ms once in a few hundred pushes, which dominated the
  // latency tail of served streams.
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    of_session* x = ss[i];
    e = launch_copy(x->mem + x->slot_off[x->cur][0], frames[i],
                    (size_t)x->H * x->W * elem_bytes(x->g.e0), st);
  }
  if (e == hipSuccess) e = launch_copy(dblk, s->host_blk_dev + (size_t)slot * s->slot_bytes, p.bytes, st);
  if (e != hipSuccess) return hip_fail("push copies", e);
  // 3. new pyramids, then the iterations of the flowing sessions
  for (int l = 1; l < L && e == hipSuccess; ++l) {
    const int ni = (int)p.items[l - 1].size();
    e = launch_reduce_batch(gg.elem(l - 1), gg.ep, (const ReduceJob*)(dblk + p.off_jobs[l - 1]),
                            (const int2*)(dblk + p.off_items[l - 1]), ni, std::min(ni, 8192), st);
  }
  int phase = 0;
  for (int l = L - 1; l >= 0 && e == hipSuccess && !flowing.empty(); --l)
    for (int k = 0; k < K && e == hipSuccess; ++k, ++phase) {
      BatchLaunch bl;
      bl.args = (const IterArgs*)(dblk + p.off_args[phase]);
      bl.tiles = (const int4*)(dblk + p.off_tiles[l]);
      // Every phase computes the tiles with an unmasked pixel only; the final phase zero-fills
      // the all-masked tiles of the caller's planes with a launch of its own.
      bl.ntiles = p.nactive[l];
      const int nzero = (l == 0 && k == K - 1) ? (int)p.tiles[l].size() - p.nactive[l] : 0;
      bl.grid = (bl.ntiles + 7) / 8 * 8;
      bl.variant = default_tile_variant((int)p.tiles[l].size());
      if (s->flags & OF_FLAG_GAUSSIAN_WINDOW) bl.variant |= kTileGauss;
      bl.masked = p.partial[l];   // only tiles with masked and unmasked pixels need the mask
      const int mode = k > 0 ? kFlowSame : (l == L - 1 ? kFlowZero : kFlowCoarse);
      if (bl.ntiles > 0) e = launch_iter_batch(gg.elem(l), bl, R, mode, st);
      if (e == hipSuccess && nzero > 0)
        e = launch_zero_tiles(bl.args, bl.tiles + bl.ntiles, nzero, TW, st);
    }
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    of_session* x = ss[i];
    if (x->has_prev && K == 0) e = launch_zero(u[i], v[i], (size_t)x->H * x->W, st);
  }
  if (e == hipSuccess) e = hipEventRecord(s->done[slot], st);
  if (e != hipSuccess) return hip_fail("push launch", e);
  s->in_use[slot] = true;
  s->next = (slot + 1) % kRing;
  // 4. the new frame becomes the previous one
  for (int i = 0; i < n; ++i) {
    of_session* x = ss[i];
    has_flow[i] = x->has_prev ? 1 : 0;
    x->has_prev = true;
    x->cur ^= 1;
  }
  return OF_OK;
}

of_status of_session_push(of_session* ss, const void* frame, float* u, float* v, void* stream,
                          int* has_flow) {
  if (!ss) return set_error("NULL session"), OF_EINVAL;
  return of_server_push(ss->server, &ss, 1, &frame, &u, &v, has_flow, stream);
}

of_status of_session_set_mask(of_session* ss, const uint8_t* mask, void* stream) {
  if (!ss) return set_error("NULL session"), OF_EINVAL;
  of_server* s = ss->server;
  std::lock_guard<std::mutex> lock(s->mu);
  DeviceGuard guard(s->device);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipDeviceSynchronize();   // pushes in flight read the old mask
  if (e != hipSuccess) return hip_fail("set_mask", e);
  if (ss->maskbuf) hipFree(ss->maskbuf);
  ss->maskbuf = nullptr;
  ss->hflags.clear();
  ss->hcut.clear();
  if (!mask) return OF_OK;
  e = prime_push_kernels(s, true);
  if (e != hipSuccess) return hip_fail("set_mask", e);
  const Geometry& g = ss->g;
  const int L = s->L, TW = strip_width_for(s->R), N = 2 * s->R + 1;
  size_t mt = 0, ft = 0;
  for (int l = 0; l < L; ++l) {
    ss->mask_off[l] = mt;
    mt += align256((size_t)g.H[l] * g.W[l]);
    for (int b = 0; b < 3; ++b) {
      ss->flag_off[b][l] = ft;
      const int TH = N * kPushBands[b];
      ft += (size_t)((g.W[l] + TW - 1) / TW) * ((g.H[l] + TH - 1) / TH);
    }
  }
  const size_t planes_at = mt;
  for (int l = 1; l < L; ++l) {
    ss->plane_off[l] = mt;
    mt += align256(4 * (size_t)g.H[l] * g.W[l] * sizeof(float));
  }
  uint8_t* mb = nullptr;
  e = hipMalloc((void**)&mb, mt);
  if (e == hipSuccess) e = hipMemcpyAsync(mb, mask, (size_t)g.H[0] * g.W[0], hipMemcpyDeviceToDevice, st);
  for (int l = 1; l < L && e == hipSuccess; ++l)
    e = launch_mask_reduce(mb + ss->mask_off[l - 1], g.H[l - 1], g.W[l - 1], mb + ss->mask_off[l],
                           g.H[l], g.W[l], st);
  // zero flow in every intermediate plane: the level-0 planes (written by earlier pushes) and
  // the planes of levels >= 1
  if (e == hipSuccess && mt > planes_at) e = hipMemsetAsync(mb + planes_at, 0, mt - planes_at, st);
  if (e == hipSuccess)
    e = hipMemsetAsync(ss->flow, 0, 4 * align256((size_t)ss->H * ss->W * sizeof(float)), st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  std::vector<uint8_t> flags(ft);
  std::vector<int2> cuts(ft, make_int2(0, 0));
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    std::vector<uint8_t> hm((size_t)g.H[l] * g.W[l]);
    e = hipMemcpy(hm.data(), mb + ss->mask_off[l], hm.size(), hipMemcpyDeviceToHost);
    for (int b = 0; b < 3 && e == hipSuccess; ++b) {
      const int TH = N * kPushBands[b];
      const std::vector<uint8_t> f = tile_flags(hm.data(), g.H[l], g.W[l], TW, TH);
      const size_t o = ss->flag_off[b][l];
      memcpy(flags.data() + o, f.data(), f.size());
      const int tx = (g.W[l] + TW - 1) / TW;
      for (size_t i = 0; i < f.size(); ++i) {
        if (f[i] != 1) continue;
        const int yy = (int)(i / tx), xx = (int)(i % tx), y0 = yy * TH;
        int ty0, th;
        band_cut(hm.data(), g.W[l], xx * TW, std::min(g.W[l], xx * TW + TW), y0,
                 std::min(g.H[l], y0 + TH), N, ty0, th);
        cuts[o + i] = make_int2(ty0, th);
      }
    }
  }
  if (e != hipSuccess) {
    if (mb) hipFree(mb);
    return hip_fail("set_mask", e);
  }
  ss->maskbuf = mb;
  ss->hflags = std::move(flags);
  ss->hcut = std::move(cuts);
  return OF_OK;
}

of_session* of_session_create(int H, int W, int levels, int radius, int iters, unsigned flags,
                              void* workspace, size_t workspace_bytes) {
  flags &= ~OF_FLAG_NO_GRAPH;
  if (!check_server_flags(flags)) return nullptr;
  if (!check_params(H, W, levels, radius, iters, flags)) return nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail("hipGetDevice", e), nullptr;
  // The registry lock is held across the open so that of_session_destroy cannot retire the
  // server in between.
  std::lock_guard<std::mutex> lock(g_hidden_mu);
  const auto key = std::make_tuple(dev, levels, radius, iters, flags);
  auto it = g_hidden.find(key);
  of_server* s;
  if (it == g_hidden.end()) {
    s = of_server_create(levels, radius, iters, flags, 0);
    if (!s) return nullptr;
    s->hidden = true;
    g_hidden[key] = s;
  } else {
    s = it->second;
  }
  return open_session(s, H, W, workspace, workspace_bytes);
}

of_status of_session_push_many(of_session* const* ss, int n, const void* const* frames,
                               float* const* u, float* const* v, int* has_flow, void* stream) {
  if (!ss || n < 1 || !ss[0]) return set_error("NULL or empty session array"), OF_EINVAL;
  return of_server_push(ss[0]->server, ss, n, frames, u, v, has_flow, stream);
}

void of_session_destroy(of_session* ss) {
  if (!ss) return;
  of_server* s = ss->server;
  if (!s->hidden) {
    of_server_close(s, ss);
    return;
  }
  std::lock_guard<std::mutex> lock(g_hidden_mu);
  of_server_close(s, ss);
  {
    if (s->sessions.empty()) {
      for (auto it = g_hidden.begin(); it != g_hidden.end(); ++it)
        if (it->second == s) {
          g_hidden.erase(it);
          break;
        }
      destroy_server(s);
    }
  }
}

void of_server_destroy(of_server* s) {
  if (!s || s->hidden) return;
  destroy_server(s);
}

}  // extern "C"
