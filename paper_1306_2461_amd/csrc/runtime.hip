// Host runtime behind the C ABI: plan validation, workspace layout and the level x iteration
// schedule of the pyramidal method (Sec. 2.4: coarsest level first from a zero field, each
// level seeding the next finer one).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/ofmi.h"
#include "kernels.h"
#include "runtime.h"

namespace ofmi {

thread_local std::string g_last_error;

void set_error(const std::string& s) { g_last_error = s; }

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool check_params(int H, int W, int levels, int radius, int iters, unsigned flags) {
  if (H < 1 || W < 1) return set_error("H and W must be >= 1"), false;
  if ((long long)H * W >= (1ll << 30)) return set_error("H * W must be below 2^30"), false;
  if (H >= (1 << 24) || W >= (1 << 24)) return set_error("H and W must be below 2^24"), false;
  if (levels < 1 || levels > OF_MAX_LEVELS) return set_error("levels out of range"), false;
  int m = H < W ? H : W, maxl = 1;
  while (m >= 2) { m >>= 1; ++maxl; }
  if (levels > maxl) return set_error("levels > 1 + floor(log2(min(H, W)))"), false;
  if (radius < 0 || radius > OF_MAX_RADIUS) return set_error("radius out of range"), false;
  if (iters < 0 || iters > OF_MAX_ITERS) return set_error("iters out of range"), false;
  if (flags & ~(OF_FLAG_FP16_STORAGE | OF_FLAG_INPUT_F32 | OF_FLAG_NO_GRAPH | OF_FLAG_NORMALIZE |
                OF_FLAG_GAUSSIAN_WINDOW | OF_FLAG_GRAPH))
    return set_error("unknown flags"), false;
  return true;
}

// Tile height (in bands of 2R+1 rows) of a plan's iteration kernel for one level: planes of
// 2^19 pixels and more take four bands (the vertical halo and the priming band amortised over
// more rows; fastest measured at 1024^2 and 2048^2), smaller ones one band (more workgroups,
// and the two-bands-per-pass variants run a one-band tile as a single trip).
int default_bands(int H, int W, int R) {
  const long long px = (long long)H * W;
  (void)R;
  return px >= (1 << 19) ? 4 : 1;
}

// Launches of about one tile per CU are latency bound and take the wide variant (shortest
// dependent path per band); launches with more tiles take the wide lean variant, whose lower
// register count lets two workgroups share a CU.
int default_tile_variant(long long ntiles) { return ntiles >= 384 ? kTileWideLean : kTileWide; }

Geometry make_geometry(int H, int W, int levels, int radius, int iters, unsigned flags) {
  Geometry g{};
  g.L = levels;
  g.R = radius;
  g.K = iters;
  g.flags = flags;
  g.H[0] = H;
  g.W[0] = W;
  for (int l = 1; l < levels; ++l) {
    g.H[l] = (g.H[l - 1] + 1) / 2;
    g.W[l] = (g.W[l - 1] + 1) / 2;
  }
  for (int l = 0; l < levels; ++l) {
    g.nb[l] = default_bands(g.H[l], g.W[l], radius);
    {
      // Variant by the level's tile count on 64-column strips at that height.  Levels of many
      // tiles, and the Gaussian-weighted window, take the batch default (wide lean, or wide
      // below 384 tiles).  With the box window (fastest measured at 1024^2 and 2048^2) levels
      // of about one tile per CU take 32-column strips: with one-band tiles two bands per pass
      // (16-column strips below 128 tiles; indices recomputed per pass otherwise), r <= 8;
      // with taller tiles, or above r = 8, one band per pass.
      const long long tx = (g.W[l] + strip_width_for(radius) - 1) / strip_width_for(radius);
      const long long th = (long long)(2 * radius + 1) * g.nb[l];
      const long long nt = tx * ((g.H[l] + th - 1) / th);
      const int v = default_tile_variant(nt);
      g.variant[l] = v;
      if (v == kTileWide && !(flags & OF_FLAG_GAUSSIAN_WINDOW)) {
        if (g.nb[l] > 1 || radius > kMaxPairRadius)
          g.variant[l] = kTileWide32;
        else
          g.variant[l] = nt < 128 ? kTileWide16x2 : kTileLean32x2;
      }
    }
  }
  g.ein = (flags & OF_FLAG_INPUT_F32) ? Elem::F32 : Elem::U8;
  g.e0 = (flags & OF_FLAG_NORMALIZE) ? Elem::F32 : g.ein;
  g.ep = (flags & OF_FLAG_FP16_STORAGE) ? Elem::F16 : Elem::F32;
  size_t off = 0;
  if (flags & OF_FLAG_NORMALIZE) {
    for (int i = 0; i < 2; ++i) {
      g.off_norm[i] = off;
      off += align256((size_t)H * W * sizeof(float));
    }
  }
  for (int l = 1; l < levels; ++l) {
    const size_t b = align256((size_t)g.H[l] * g.W[l] * elem_bytes(g.ep));
    g.off_p1[l] = off;
    off += b;
    g.off_p2[l] = off;
    off += b;
  }
  const size_t fb = align256((size_t)H * W * sizeof(float));
  for (int i = 0; i < 4; ++i) {
    g.off_flow[i] = off;
    off += fb;
  }
  g.bytes = off;
  return g;
}

Elem Geometry::elem(int l) const { return l == 0 ? e0 : ep; }

hipError_t KernelTimer::begin(hipStream_t s, hipEvent_t* a) {
  *a = nullptr;
  if (!on) return hipSuccess;
  if (pool.empty()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pool.push_back(e);
  }
  *a = pool.back();
  pool.pop_back();
  return hipEventRecord(*a, s);
}

hipError_t KernelTimer::end(hipStream_t s, hipEvent_t a, int kernel, double units, double bytes,
                            long long launches) {
  if (!on || !a) return hipSuccess;
  hipEvent_t b;
  if (pool.empty()) {
    hipError_t r = hipEventCreate(&b);
    if (r != hipSuccess) return r;
  } else {
    b = pool.back();
    pool.pop_back();
  }
  recs.push_back({kernel, a, b, units, bytes, launches});
  return hipEventRecord(b, s);
}

hipError_t KernelTimer::read(int kernel, double* ms, long long* n, double* units, double* bytes) {
  double tms = 0, tu = 0, tb = 0;
  long long cnt = 0;
  std::vector<Rec> keep;
  for (const Rec& r : recs) {
    if (r.kernel != kernel) {
      keep.push_back(r);
      continue;
    }
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return e;
    float f = 0.f;
    e = hipEventElapsedTime(&f, r.a, r.b);
    if (e != hipSuccess) return e;
    tms += f;
    tu += r.units;
    tb += r.bytes;
    cnt += r.launches;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.swap(keep);
  if (ms) *ms = tms;
  if (n) *n = cnt;
  if (units) *units = tu;
  if (bytes) *bytes = tb;
  return hipSuccess;
}

void GraphCache::clear() {
  for (Entry& e : entries) hipGraphExecDestroy(e.exec);
  entries.clear();
}

GraphCache::~GraphCache() {
  clear();
  if (cap) hipStreamDestroy(cap);
}

KernelTimer::~KernelTimer() {
  for (const Rec& r : recs) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) hipEventDestroy(e);
}

// Window taps and launch variant of one iteration: the Gaussian-weighted window
// (OF_FLAG_GAUSSIAN_WINDOW) fills the taps g(d) = exp(-d^2 / (2 sigma^2)), sigma = r/2,
// d = -r..r, and marks the variant.
void gaussian_taps(float* taps, int R) {
  for (int q = 0; q <= 2 * R; ++q) {
    const double d = q - R;
    taps[q] = R == 0 ? 1.0f : (float)std::exp(-2.0 * d * d / ((double)R * R));
  }
}

std::vector<uint8_t> tile_flags(const uint8_t* m, int H, int W, int TW, int TH) {
  const int tx = (W + TW - 1) / TW, ty = (H + TH - 1) / TH;
  std::vector<uint8_t> f((size_t)tx * ty);
  for (int by = 0; by < ty; ++by)
    for (int bx = 0; bx < tx; ++bx) {
      int on = 0, total = 0;
      for (int y = by * TH; y < std::min(H, (by + 1) * TH); ++y)
        for (int x = bx * TW; x < std::min(W, (bx + 1) * TW); ++x) {
          on += m[(size_t)y * W + x] != 0;
          ++total;
        }
      f[(size_t)by * tx + bx] = on == 0 ? 0 : (on == total ? 2 : 1);
    }
  return f;
}

void band_cut(const uint8_t* m, int W, int c0, int c1, int y0, int e, int N, int& ty0, int& th) {
  int r0 = e, r1 = y0;   // rows [r0, r1) hold an unmasked pixel
  for (int y = y0; y < e; ++y) {
    const uint8_t* row = m + (size_t)y * W;
    bool any = false;
    for (int c = c0; c < c1 && !any; ++c) any = row[c] != 0;
    if (any) {
      if (r0 == e) r0 = y;
      r1 = y + 1;
    }
  }
  if (r0 >= r1) {   // nothing unmasked: an empty cut
    ty0 = y0;
    th = 0;
    return;
  }
  ty0 = y0 + (r0 - y0) / N * N;
  th = ((r1 - 1 - ty0) / N + 1) * N;
}

int window_variant(const Geometry& g, int l, IterArgs& a) {
  if (!(g.flags & OF_FLAG_GAUSSIAN_WINDOW)) return g.variant[l];
  gaussian_taps(a.taps, g.R);
  return g.variant[l] | kTileGauss;
}

// Enqueue the whole method for one pair: pyramid then levels x iterations.
hipError_t enqueue_pair(const Geometry& g, char* ws, const void* I1, const void* I2, float* u,
                        float* v, hipStream_t s, KernelTimer* t) {
  const size_t n0 = (size_t)g.H[0] * g.W[0];
  if (g.bcount) {
    hipError_t e = launch_zero_count(g.bcount, s);
    if (e != hipSuccess) return e;
  }
  if (g.K == 0) {
    hipError_t e = launch_zero(u, v, n0, s);
    if (e == hipSuccess && g.bcount) e = launch_count_at_most(u, (long long)n0, g.bthr, g.bcount, s);
    return e;
  }
  const void* P1[OF_MAX_LEVELS];
  const void* P2[OF_MAX_LEVELS];
  P1[0] = I1;
  P2[0] = I2;
  if (g.flags & OF_FLAG_NORMALIZE) {
    float* n1 = (float*)(ws + g.off_norm[0]);
    float* n2 = (float*)(ws + g.off_norm[1]);
    hipError_t e = launch_normalize(g.ein, I1, n1, g.H[0], g.W[0], OF_NORMALIZE_RADIUS,
                                    OF_NORMALIZE_EPS, s);
    if (e == hipSuccess)
      e = launch_normalize(g.ein, I2, n2, g.H[0], g.W[0], OF_NORMALIZE_RADIUS, OF_NORMALIZE_EPS, s);
    if (e != hipSuccess) return e;
    P1[0] = n1;
    P2[0] = n2;
  }
  for (int l = 1; l < g.L; ++l) {
    P1[l] = ws + g.off_p1[l];
    P2[l] = ws + g.off_p2[l];
  }
  // Pyramid: runs of 2 or 3 levels whose first output plane has at most 2^20 pixels take one
  // fused chain launch each, other levels one reduction each (identical bits either way).
  hipEvent_t span = nullptr;
  double span_units = 0, span_bytes = 0;
  long long span_launches = 0;
  if (t && t->per_level() && g.L > 1) {
    hipError_t e = t->begin(s, &span);
    if (e != hipSuccess) return e;
  }
  for (int l = 1; l < g.L;) {
    const int rest = g.L - l;
    const int D = (rest >= 2 && (long long)g.H[l] * g.W[l] <= (1ll << 20)) ? (rest >= 3 ? 3 : 2) : 1;
    hipEvent_t ev;
    hipError_t e = t && t->per_launch() ? t->begin(s, &ev) : hipSuccess;
    if (e == hipSuccess) {
      if (D == 1) {
        e = launch_reduce(g.elem(l - 1), g.ep, P1[l - 1], P2[l - 1], g.H[l - 1], g.W[l - 1],
                          (void*)P1[l], (void*)P2[l], g.H[l], g.W[l], s);
      } else {
        ReduceChain c{};
        c.in[0] = P1[l - 1];
        c.in[1] = P2[l - 1];
        for (int d = 0; d <= D; ++d) {
          c.H[d] = g.H[l - 1 + d];
          c.W[d] = g.W[l - 1 + d];
        }
        for (int d = 1; d <= D; ++d) {
          c.out[0][d - 1] = (void*)P1[l - 1 + d];
          c.out[1][d - 1] = (void*)P2[l - 1 + d];
        }
        c.D = D;
        e = launch_reduce_chain(g.elem(l - 1), g.ep, c, s);
      }
    }
    if (e == hipSuccess && t) {
      // algorithmic: each input plane read once, each output plane written once
      double no = 0;
      for (int d = 0; d < D; ++d) no += (double)g.H[l + d] * g.W[l + d];
      const double ni = (double)g.H[l - 1] * g.W[l - 1];
      const double by = 2 * (ni * elem_bytes(g.elem(l - 1)) + no * elem_bytes(g.ep));
      if (t->per_launch()) e = t->end(s, ev, OF_KERNEL_REDUCE, 2 * no, by);
      span_units += 2 * no;
      span_bytes += by;
      ++span_launches;
    }
    if (e != hipSuccess) return e;
    l += D;
  }
  if (span) {
    hipError_t e = t->end(s, span, OF_KERNEL_REDUCE, span_units, span_bytes, span_launches);
    if (e != hipSuccess) return e;
  }
  float* fu[2] = {(float*)(ws + g.off_flow[0]), (float*)(ws + g.off_flow[1])};
  float* fv[2] = {(float*)(ws + g.off_flow[2]), (float*)(ws + g.off_flow[3])};
  const float* cu = nullptr;
  const float* cv = nullptr;
  int cH = 0, cW = 0, buf = 0;
  for (int l = g.L - 1; l >= 0; --l) {
    hipEvent_t lspan = nullptr;
    if (t && t->per_level()) {
      hipError_t e = t->begin(s, &lspan);
      if (e != hipSuccess) return e;
    }
    for (int k = 0; k < g.K; ++k) {
      IterArgs a{};
      a.I1 = P1[l];
      a.I2 = P2[l];
      a.H = g.H[l];
      a.W = g.W[l];
      a.uin = cu;
      a.vin = cv;
      a.Hc = cH;
      a.Wc = cW;
      a.mode = k > 0 ? kFlowSame : (l == g.L - 1 ? kFlowZero : kFlowCoarse);
      a.mask = g.mask[l];
      a.tiles = g.tflags[l];
      const bool last = (l == 0 && k == g.K - 1);
      a.uout = last ? u : fu[buf];
      a.vout = last ? v : fv[buf];
      if (last) {
        a.bthr = g.bthr;
        a.bcount = g.bcount;
      }
      hipEvent_t ev;
      hipError_t e = t && t->per_launch() ? t->begin(s, &ev) : hipSuccess;
      const int variant = window_variant(g, l, a);
      if (e == hipSuccess) e = launch_iter(g.elem(l), a, g.R, g.nb[l], variant, s);
      if (e == hipSuccess && t && t->per_launch()) {
        const double n = (double)a.H * a.W;
        e = t->end(s, ev, OF_KERNEL_ITERATE, n, n * (2.0 * elem_bytes(g.elem(l)) + 16.0));
      }
      if (e != hipSuccess) return e;
      cu = a.uout;
      cv = a.vout;
      cH = a.H;
      cW = a.W;
      buf ^= 1;
    }
    if (lspan) {
      const double n = (double)g.H[l] * g.W[l] * g.K;
      hipError_t e = t->end(s, lspan, OF_KERNEL_LEVEL(l), n,
                            n * (2.0 * elem_bytes(g.elem(l)) + 16.0), g.K);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace ofmi

using namespace ofmi;

struct of_plan {
  Geometry g;
  char* ws;
  bool owns_ws;
  int device;
  uint8_t* maskbuf = nullptr;   // mask pyramid (of_plan_set_mask), all levels
  uint8_t* tflags = nullptr;    // iteration-tile flags of all levels (capacity: one band per tile)
  size_t tf_off[OF_MAX_LEVELS] = {};
  std::vector<uint8_t> hmask[OF_MAX_LEVELS];   // host copy of the mask pyramid
  KernelTimer timer;
  GraphCache graphs;
};

namespace {

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

}  // namespace

extern "C" {

size_t of_plan_workspace_bytes(int H, int W, int levels, int radius, int iters, unsigned flags) {
  if (!check_params(H, W, levels, radius, iters, flags)) return 0;
  return make_geometry(H, W, levels, radius, iters, flags).bytes;
}

of_plan* of_plan_create_ex(int H, int W, int levels, int radius, int iters, unsigned flags,
                           void* workspace, size_t workspace_bytes) {
  if (!check_params(H, W, levels, radius, iters, flags)) return nullptr;
  Geometry g = make_geometry(H, W, levels, radius, iters, flags);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    hip_fail("hipGetDevice", e);
    return nullptr;
  }
  char* ws = (char*)workspace;
  bool owns = false;
  if (ws) {
    if (workspace_bytes < g.bytes) {
      set_error("workspace smaller than of_plan_workspace_bytes()");
      return nullptr;
    }
    if ((uintptr_t)ws & 255) {
      set_error("workspace must be 256-byte aligned");
      return nullptr;
    }
  } else {
    e = hipMalloc((void**)&ws, g.bytes);
    if (e != hipSuccess) {
      hip_fail("hipMalloc(workspace)", e);
      return nullptr;
    }
    owns = true;
  }
  of_plan* p = new of_plan{g, ws, owns, dev, {}, {}};
  return p;
}

of_plan* of_plan_create(int H, int W, int levels, int radius, int iters) {
  return of_plan_create_ex(H, W, levels, radius, iters, 0u, nullptr, 0);
}

of_status of_compute(of_plan* p, const void* I1, const void* I2, float* u, float* v,
                     void* stream) {
  if (!p) return set_error("NULL plan"), OF_EINVAL;
  if (!I1 || !I2 || !u || !v) return set_error("NULL frame or output pointer"), OF_EINVAL;
  if (u == v) return set_error("u and v must be distinct planes"), OF_EINVAL;
  if (((uintptr_t)u | (uintptr_t)v) & 3) return set_error("u, v must be 4-byte aligned"), OF_EINVAL;
  if ((p->g.flags & OF_FLAG_INPUT_F32) && (((uintptr_t)I1 | (uintptr_t)I2) & 3))
    return set_error("float32 frames must be 4-byte aligned"), OF_EINVAL;
  DeviceGuard guard(p->device);
  hipError_t e;
  if (p->timer.on || (p->g.flags & OF_FLAG_NO_GRAPH) || !(p->g.flags & OF_FLAG_GRAPH)) {
    e = enqueue_pair(p->g, p->ws, I1, I2, u, v, (hipStream_t)stream, &p->timer);
  } else {
    const std::vector<uintptr_t> key = {(uintptr_t)I1, (uintptr_t)I2, (uintptr_t)u, (uintptr_t)v};
    e = p->graphs.run(key, (hipStream_t)stream, [&](hipStream_t cs) {
      return enqueue_pair(p->g, p->ws, I1, I2, u, v, cs, nullptr);
    });
  }
  if (e != hipSuccess) return hip_fail("kernel launch", e);
  return OF_OK;
}

}  // extern "C"

namespace {

// Device scratch of of_compute_noalloc: a file-scope array of fixed size (each device that
// runs the library holds one until the process ends).  Host code never uses the array's name
// as an address: the device address of each device's copy comes from hipGetSymbolAddress,
// taken once per device with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)OF_NOALLOC_SCRATCH_MIB << 20;
__device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (set up on the first call per device).
hipError_t scratch_for(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t of_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

of_status of_compute_noalloc(int H, int W, int levels, int radius, int iters, unsigned flags,
                             const void* I1, const void* I2, float* u, float* v, void* stream) {
  if (flags & (OF_FLAG_GRAPH | OF_FLAG_NO_GRAPH))
    return set_error("of_compute_noalloc launches eagerly: graph flags are not accepted"), OF_EINVAL;
  if (!check_params(H, W, levels, radius, iters, flags)) return OF_EINVAL;
  if (!I1 || !I2 || !u || !v) return set_error("NULL frame or output pointer"), OF_EINVAL;
  if (u == v) return set_error("u and v must be distinct planes"), OF_EINVAL;
  if (((uintptr_t)u | (uintptr_t)v) & 3) return set_error("u, v must be 4-byte aligned"), OF_EINVAL;
  if ((flags & OF_FLAG_INPUT_F32) && (((uintptr_t)I1 | (uintptr_t)I2) & 3))
    return set_error("float32 frames must be 4-byte aligned"), OF_EINVAL;
  const Geometry g = make_geometry(H, W, levels, radius, iters, flags);
  if (g.bytes > kNoallocScratchBytes)
    return set_error("of_compute_noalloc: this frame size needs " + std::to_string(g.bytes) +
                     " bytes of scratch, more than the library's " +
                     std::to_string(kNoallocScratchBytes)),
           OF_ENOMEM;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  char* ws = nullptr;
  if (e == hipSuccess) e = scratch_for(dev, &ws);
  if (e != hipSuccess) return hip_fail("noalloc scratch", e);
  e = enqueue_pair(g, ws, I1, I2, u, v, (hipStream_t)stream, nullptr);
  if (e != hipSuccess) return hip_fail("kernel launch", e);
  return OF_OK;
}

void of_plan_destroy(of_plan* p) {
  if (!p) return;
  DeviceGuard guard(p->device);
  hipDeviceSynchronize();
  p->graphs.clear();
  if (p->owns_ws) hipFree(p->ws);
  if (p->maskbuf) hipFree(p->maskbuf);
  if (p->tflags) hipFree(p->tflags);
  delete p;
}

const char* of_last_error(void) { return g_last_error.c_str(); }

namespace {

// Tile count of level l at one band per tile on the narrowest strips (16 columns).
size_t tile_capacity(const Geometry& g, int l) {
  const size_t tx = (g.W[l] + 15) / 16;
  return tx * ((g.H[l] + 2 * g.R) / (2 * g.R + 1));
}

// Flags of level l's iteration tiles for its current tile height, from the host mask copy,
// uploaded to the plan's flag buffer (synchronous copy: outside graph capture only).
hipError_t upload_tile_flags(of_plan* p, int l) {
  Geometry& g = p->g;
  const int TW = tile_width(g.variant[l], g.R), TH = (2 * g.R + 1) * g.nb[l];
  const std::vector<uint8_t> f = tile_flags(p->hmask[l].data(), g.H[l], g.W[l], TW, TH);
  g.tflags[l] = p->tflags + p->tf_off[l];
  return hipMemcpy(p->tflags + p->tf_off[l], f.data(), f.size(), hipMemcpyHostToDevice);
}

hipError_t upload_all_tile_flags(of_plan* p) {
  hipError_t e = hipSuccess;
  if (!p->g.mask[0]) return e;
  for (int l = 0; l < p->g.L && e == hipSuccess; ++l) e = upload_tile_flags(p, l);
  return e;
}

}  // namespace

of_status of_plan_set_mask(of_plan* p, const uint8_t* mask, void* stream) {
  if (!p) return set_error("NULL plan"), OF_EINVAL;
  DeviceGuard guard(p->device);
  hipStream_t s = (hipStream_t)stream;
  Geometry& g = p->g;
  hipError_t e = hipStreamSynchronize(s);   // graphs in flight may still read the old masks
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail("set_mask", e);
  p->graphs.clear();
  if (!mask) {
    for (int l = 0; l < g.L; ++l) g.mask[l] = g.tflags[l] = nullptr;
    return OF_OK;
  }
  size_t off[OF_MAX_LEVELS], total = 0, ftotal = 0;
  for (int l = 0; l < g.L; ++l) {
    off[l] = total;
    total += align256((size_t)g.H[l] * g.W[l]);
    p->tf_off[l] = ftotal;
    ftotal += align256(tile_capacity(g, l));
  }
  if (!p->maskbuf) {
    e = hipMalloc((void**)&p->maskbuf, total);
    if (e == hipSuccess) e = hipMalloc((void**)&p->tflags, ftotal);
    if (e != hipSuccess) {
      if (p->maskbuf) hipFree(p->maskbuf);
      p->maskbuf = nullptr;
      p->tflags = nullptr;
      set_error(std::string("mask allocation: ") + hipGetErrorString(e));
      return OF_ENOMEM;
    }
  }
  e = hipMemcpyAsync(p->maskbuf, mask, (size_t)g.H[0] * g.W[0], hipMemcpyDeviceToDevice, s);
  for (int l = 1; l < g.L && e == hipSuccess; ++l)
    e = launch_mask_reduce(p->maskbuf + off[l - 1], g.H[l - 1], g.W[l - 1], p->maskbuf + off[l],
                           g.H[l], g.W[l], s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (int l = 0; l < g.L && e == hipSuccess; ++l) {
    p->hmask[l].resize((size_t)g.H[l] * g.W[l]);
    e = hipMemcpy(p->hmask[l].data(), p->maskbuf + off[l], p->hmask[l].size(), hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) {
    for (int l = 0; l < g.L; ++l) g.mask[l] = g.tflags[l] = nullptr;
    return hip_fail("set_mask", e);
  }
  for (int l = 0; l < g.L; ++l) g.mask[l] = p->maskbuf + off[l];
  e = upload_all_tile_flags(p);
  if (e != hipSuccess) {
    for (int l = 0; l < g.L; ++l) g.mask[l] = g.tflags[l] = nullptr;
    return hip_fail("set_mask tile flags", e);
  }
  return OF_OK;
}

int of_levels_for_displacement(float dmax, int H, int W) {
  if (H < 1 || W < 1 || !(dmax >= 0.f) || !(dmax < 1e30f)) return 0;
  int m = H < W ? H : W, maxl = 1;
  while (m >= 2) { m >>= 1; ++maxl; }
  if (maxl > OF_MAX_LEVELS) maxl = OF_MAX_LEVELS;
  int L = 1;
  // eq. 1: dmax / 2^(L-1) < 3 px, evaluated in double (exact for the powers of two)
  while (L < maxl && (double)dmax / (double)(1ll << (L - 1)) >= 3.0) ++L;
  return L;
}

of_status of_plan_set_bubble(of_plan* p, const float* threshold, unsigned long long* count) {
  if (!p) return set_error("NULL plan"), OF_EINVAL;
  if ((threshold == nullptr) != (count == nullptr))
    return set_error("threshold and count are set or removed together"), OF_EINVAL;
  if (((uintptr_t)threshold & 3) || ((uintptr_t)count & 7))
    return set_error("misaligned threshold or count"), OF_EINVAL;
  DeviceGuard guard(p->device);
  hipDeviceSynchronize();   // captured schedules hold the old pointers
  p->graphs.clear();
  p->g.bthr = threshold;
  p->g.bcount = count;
  return OF_OK;
}

of_status of_plan_get_config(const of_plan* p, int* bands, int* variant) {
  if (!p || !bands || !variant) return set_error("NULL argument"), OF_EINVAL;
  for (int l = 0; l < p->g.L; ++l) {
    bands[l] = p->g.nb[l];
    variant[l] = p->g.variant[l];
  }
  return OF_OK;
}

of_status of_plan_set_config(of_plan* p, const int* bands, const int* variant) {
  if (!p || !bands || !variant) return set_error("NULL argument"), OF_EINVAL;
  for (int l = 0; l < p->g.L; ++l) {
    if (bands[l] < 1 || bands[l] > 64) return set_error("bands out of range"), OF_EINVAL;
    if (variant[l] < kTileNarrow || variant[l] >= kTileVariants)
      return set_error("tile variant out of range"), OF_EINVAL;
    if (variant[l] > kTileWideLean && (p->g.flags & OF_FLAG_GAUSSIAN_WINDOW))
      return set_error("narrow-strip variants apply to the box window only"), OF_EINVAL;
    if (!tile_variant_valid(variant[l], p->g.R, p->g.flags & OF_FLAG_GAUSSIAN_WINDOW))
      return set_error("two-bands-per-pass variants take r <= 8"), OF_EINVAL;
  }
  DeviceGuard guard(p->device);
  hipDeviceSynchronize();
  p->graphs.clear();
  for (int l = 0; l < p->g.L; ++l) {
    p->g.nb[l] = bands[l];
    p->g.variant[l] = variant[l];
  }
  hipError_t e = upload_all_tile_flags(p);
  if (e != hipSuccess) return hip_fail("tile flags", e);
  return OF_OK;
}

of_status of_plan_autotune(of_plan* p, const void* I1, const void* I2, float* u, float* v,
                           void* stream, int reps) {
  if (!p || !I1 || !I2 || !u || !v || u == v) return set_error("bad argument"), OF_EINVAL;
  if (reps < 1) reps = 1;
  DeviceGuard guard(p->device);
  hipStream_t s = (hipStream_t)stream;
  Geometry& g = p->g;
  const bool was_on = p->timer.on;
  const int was_mode = p->timer.mode;
  p->timer.on = true;
  p->timer.mode = OF_TIMING_LAUNCH;
  static const int kBands[] = {1, 2, 3, 4, 8};
  hipError_t e = hipSuccess;
  for (int l = 0; l < g.L && e == hipSuccess && g.K > 0; ++l) {
    double best = 1e30;
    int bnb = g.nb[l];
    int bw = g.variant[l];
    for (int nb : kBands) {
      if (nb > 1 && (2 * g.R + 1) * nb > 2 * g.H[l]) continue;
      for (int w = kTileNarrow; w < kTileVariants; ++w) {
        if (!tile_variant_valid(w, g.R, g.flags & OF_FLAG_GAUSSIAN_WINDOW)) continue;
        g.nb[l] = nb;
        g.variant[l] = w;
        if (g.mask[l]) e = upload_tile_flags(p, l);
        if (e != hipSuccess) break;
        double tl = 1e30;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
          e = enqueue_pair(g, p->ws, I1, I2, u, v, s, &p->timer);
          if (e == hipSuccess) e = hipStreamSynchronize(s);
          if (e != hipSuccess) break;
          // launch k of level l is iteration launch (L-1-l)*K + k of the run
          const int first = (g.L - 1 - l) * g.K;
          int idx = 0;
          double sum = 0;
          for (const KernelTimer::Rec& rc : p->timer.recs) {
            if (rc.kernel != OF_KERNEL_ITERATE) continue;
            if (idx >= first && idx < first + g.K) {
              float ms = 0.f;
              hipEventElapsedTime(&ms, rc.a, rc.b);
              sum += ms;
            }
            ++idx;
          }
          double d;
          long long n;
          p->timer.read(OF_KERNEL_ITERATE, &d, &n, &d, &d);
          p->timer.read(OF_KERNEL_REDUCE, &d, &n, &d, &d);
          if (r > 0) tl = tl < sum ? tl : sum;
        }
        if (tl < best) {
          best = tl;
          bnb = nb;
          bw = w;
        }
      }
    }
    g.nb[l] = bnb;
    g.variant[l] = bw;
    if (e == hipSuccess && g.mask[l]) e = upload_tile_flags(p, l);
  }
  p->timer.on = was_on;
  p->timer.mode = was_mode;
  hipDeviceSynchronize();
  p->graphs.clear();
  if (e != hipSuccess) return hip_fail("autotune", e);
  return OF_OK;
}

of_status of_plan_set_timing(of_plan* p, int enable) {
  if (!p) return set_error("NULL plan"), OF_EINVAL;
  if (enable < 0 || enable > OF_TIMING_LEVEL) return set_error("unknown timing mode"), OF_EINVAL;
  p->timer.on = enable != 0;
  if (enable) p->timer.mode = enable;
  return OF_OK;
}

of_status of_plan_read_timing(of_plan* p, int kernel, double* total_ms, long long* launches,
                              double* units, double* bytes) {
  if (!p) return set_error("NULL plan"), OF_EINVAL;
  if (kernel != OF_KERNEL_ITERATE && kernel != OF_KERNEL_REDUCE &&
      !(kernel >= OF_KERNEL_LEVEL(0) && kernel < OF_KERNEL_LEVEL(OF_MAX_LEVELS)))
    return set_error("unknown kernel id"), OF_EINVAL;
  DeviceGuard guard(p->device);
  hipError_t e = p->timer.read(kernel, total_ms, launches, units, bytes);
  if (e != hipSuccess) return hip_fail("timing events", e);
  return OF_OK;
}

of_status of_debug_stage(of_plan* p, int stage, int level, const void* const* in,
                         void* const* out, void* stream) {
  if (!p || !in || !out) return set_error("NULL argument"), OF_EINVAL;
  const Geometry& g = p->g;
  DeviceGuard guard(p->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (stage == OF_STAGE_REDUCE) {
    if (level < 0 || level >= g.L - 1) return set_error("reduce level out of range"), OF_EINVAL;
    if (!in[0] || !out[0]) return set_error("NULL plane"), OF_EINVAL;
    e = launch_reduce(g.elem(level), g.ep, in[0], nullptr, g.H[level], g.W[level], out[0],
                      nullptr, g.H[level + 1], g.W[level + 1], s);
  } else if (stage == OF_STAGE_ITERATE) {
    if (level < 0 || level >= g.L) return set_error("level out of range"), OF_EINVAL;
    for (int i = 0; i < 4; ++i)
      if (!in[i]) return set_error("NULL input plane"), OF_EINVAL;
    if (!out[0] || !out[1] || out[0] == out[1]) return set_error("bad output planes"), OF_EINVAL;
    IterArgs a{};
    a.I1 = in[0];
    a.I2 = in[1];
    a.uin = (const float*)in[2];
    a.vin = (const float*)in[3];
    a.uout = (float*)out[0];
    a.vout = (float*)out[1];
    a.H = g.H[level];
    a.W = g.W[level];
    a.mode = kFlowSame;
    const int variant = window_variant(g, level, a);
    e = launch_iter(g.elem(level), a, g.R, g.nb[level], variant, s);
  } else {
    return set_error("unknown stage"), OF_EINVAL;
  }
  if (e != hipSuccess) return hip_fail("kernel launch", e);
  return OF_OK;
}

}  // extern "C"
