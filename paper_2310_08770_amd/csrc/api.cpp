// Host side of libccpt: argument checking, reference spectra, DFT tables,
// workspaces, the per-size launch sequence, graph capture and tuning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "tables.h"

using namespace ccpt;

namespace {

bool supported_size(int n) {
  if (n < 16 || n > 512 || (n & 1)) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

struct SizeTables {
  float2* tw = nullptr;  // N
  void* ky = nullptr;
  void* wb = nullptr;
  int Mp = 0;
};

struct Ref {
  int n = 0;
  float2* spec = nullptr;  // conj F[B], N x (N/2+1)
  float* img = nullptr;    // E as float (N x N), kept for the CC-SN chain rule
};

struct Schedule {
  int chunk = 0;  // frames per launch chunk (0 = default)
};

struct GraphKey {
  std::vector<int> sig;  // group sizes and counts
  const void* out;
  hipStream_t stream;
  bool operator<(const GraphKey& o) const {
    return std::tie(sig, out, stream) < std::tie(o.sig, o.out, o.stream);
  }
};

}  // namespace

struct ccpt_ctx {
  int device = 0;
  ccpt_options o{};
  int M = 0, c = 0;
  std::map<int, SizeTables> tables;
  std::vector<Ref> refs;
  std::map<int, Schedule> sched;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // descriptors
  FrameDesc* d_desc = nullptr;
  FrameDesc* h_desc = nullptr;
  size_t desc_cap = 0;
  std::vector<FrameDesc> last_desc;
  hipEvent_t desc_evt = nullptr;
  // captured graphs
  std::map<GraphKey, hipGraphExec_t> graphs;
  // errors
  int last_code = CCPT_OK;
  std::string last_msg;
};

namespace {

int fail(ccpt_ctx* ctx, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(ccpt_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_code = code;
    ctx->last_msg = buf;
  }
  return code;
}

#define HIP_CHECK(ctx, call)                                                               \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, CCPT_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

int set_device(ccpt_ctx* ctx) {
  HIP_CHECK(ctx, hipSetDevice(ctx->device));
  return CCPT_OK;
}

double step_limit(const ccpt_ctx* ctx) {
  const double grid = 1.0 / ctx->o.upsample;
  // split-precision grids locate the maximum less exactly than one grid step
  return ctx->o.precision == CCPT_PREC_FP32 ? grid : std::max(grid, kSplitStepLimit);
}

int ensure_tables(ccpt_ctx* ctx, int n) {
  if (ctx->tables.count(n)) return CCPT_OK;
  SizeTables t;
  HostTables h = build_tables(n, ctx->o.upsample, ctx->M, ctx->c, ctx->o.precision);
  t.Mp = h.Mp;
  HIP_CHECK(ctx, hipMalloc(&t.tw, h.tw.size() * sizeof(float2)));
  HIP_CHECK(ctx, hipMemcpy(t.tw, h.tw.data(), h.tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_CHECK(ctx, hipMalloc(&t.ky, h.ky.size()));
  HIP_CHECK(ctx, hipMemcpy(t.ky, h.ky.data(), h.ky.size(), hipMemcpyHostToDevice));
  HIP_CHECK(ctx, hipMalloc(&t.wb, h.wb.size()));
  HIP_CHECK(ctx, hipMemcpy(t.wb, h.wb.data(), h.wb.size(), hipMemcpyHostToDevice));
  ctx->tables[n] = t;
  return CCPT_OK;
}

// Captured graphs bake in workspace and descriptor addresses: drop them
// whenever either is reallocated.
void drop_graphs(ccpt_ctx* ctx) {
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
}

int ensure_ws(ccpt_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return CCPT_OK;
  drop_graphs(ctx);
  if (ctx->ws) {
    HIP_CHECK(ctx, hipDeviceSynchronize());
    HIP_CHECK(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(ctx, CCPT_E_NOMEM, "workspace of %zu bytes", bytes);
  }
  ctx->ws_bytes = bytes;
  return CCPT_OK;
}

size_t frame_ws_bytes(int n) {
  const size_t spec = (size_t)n * (n / 2 + 1) * sizeof(float2);
  return 2 * spec + sizeof(FrameState);
}

int default_chunk(int n) {
  // keep the chunk's two spectra well inside the 256 MB Infinity Cache
  const size_t budget = (size_t)192 << 20;
  int c = (int)(budget / frame_ws_bytes(n));
  return std::max(1, std::min(c, 4096));
}

int chunk_for(const ccpt_ctx* ctx, int n) {
  auto it = ctx->sched.find(n);
  if (it != ctx->sched.end() && it->second.chunk > 0) return it->second.chunk;
  return default_chunk(n);
}

// Carves the workspace for a chunk of `chunk` frames of size n.
void carve(ccpt_ctx* ctx, int n, int chunk, float2*& T, float2*& X, FrameState*& st) {
  const size_t spec = (size_t)n * (n / 2 + 1);
  T = (float2*)ctx->ws;
  X = T + spec * chunk;
  st = (FrameState*)(X + spec * chunk);
}

int check_image(ccpt_ctx* ctx, const void* data, int ny, int nx, int pitch, int dtype,
                const char* what, int idx) {
  if (!data) return fail(ctx, CCPT_E_INVALID, "%s %d: null data", what, idx);
  if (dtype != CCPT_U16 && dtype != CCPT_F32)
    return fail(ctx, CCPT_E_INVALID, "%s %d: unknown dtype %d", what, idx, dtype);
  if (ny <= 0 || nx <= 0 || pitch < nx)
    return fail(ctx, CCPT_E_INVALID, "%s %d: bad shape %dx%d pitch %d", what, idx, ny, nx, pitch);
  if (ny != nx || !supported_size(nx))
    return fail(ctx, CCPT_E_UNSUPPORTED, "%s %d: %dx%d is not a supported square size", what,
                idx, ny, nx);
  const size_t align = dtype == CCPT_U16 ? 2 : 4;
  if ((uintptr_t)data % align)
    return fail(ctx, CCPT_E_INVALID, "%s %d: misaligned data", what, idx);
  return CCPT_OK;
}

GroupParams base_params(ccpt_ctx* ctx, int n) {
  GroupParams g{};
  g.tw = ctx->tables[n].tw;
  g.mode = ctx->o.mode;
  g.eps = (float)ctx->o.eps;
  g.u = ctx->o.upsample;
  g.M = ctx->M;
  g.c = ctx->c;
  g.newton_iters = ctx->o.newton_iters;
  g.half_window = 0.5 * ctx->o.window;
  return g;
}

// Launches the whole tracking sequence for one size group, chunk by chunk.
int run_group(ccpt_ctx* ctx, int n, const FrameDesc* d_desc, int first, int count,
              ccpt_result* out, hipStream_t s) {
  const int chunk = std::min(count, chunk_for(ctx, n));
  SizeTables& t = ctx->tables[n];
  UpdftTables ut{t.ky, t.wb, t.Mp, ctx->o.precision};
  for (int c0 = 0; c0 < count; c0 += chunk) {
    GroupParams g = base_params(ctx, n);
    g.desc = d_desc;
    g.first = first + c0;
    g.count = std::min(chunk, count - c0);
    g.out = out;
    carve(ctx, n, chunk, g.T, g.X, g.st);
    if (launch_xcorr(n, g, s, 0)) return fail(ctx, CCPT_E_HIP, "correlation launch failed");
    if (launch_updft(n, g, ut, s)) return fail(ctx, CCPT_E_HIP, "upsampled DFT launch failed");
    if (launch_newton(n, g, step_limit(ctx), s))
      return fail(ctx, CCPT_E_HIP, "Newton launch failed");
  }
  return CCPT_OK;
}

}  // namespace

// ===================================================================== ABI

extern "C" {

void ccpt_default_options(ccpt_options* o) {
  if (!o) return;
  o->mode = CCPT_MODE_CCU;
  o->eps = 200.0;
  o->upsample = 100;
  o->window = 1.5;
  o->precision = CCPT_PREC_FP32;
  o->newton_iters = 3;
  o->flags = 0;
}

const char* ccpt_status_string(int code) {
  switch (code) {
    case CCPT_OK: return "ok";
    case CCPT_E_INVALID: return "invalid argument";
    case CCPT_E_UNSUPPORTED: return "unsupported frame size";
    case CCPT_E_NOREF: return "no reference for this id";
    case CCPT_E_HIP: return "HIP runtime error";
    case CCPT_E_NONPOSITIVE_REF: return "CC-SN reference has E + eps <= 0";
    case CCPT_E_NOMEM: return "out of memory";
  }
  return "unknown status";
}

int ccpt_last_error(const ccpt_ctx* ctx, char* buf, size_t len) {
  if (!ctx) return CCPT_E_INVALID;
  if (buf && len) {
    size_t k = std::min(len - 1, ctx->last_msg.size());
    memcpy(buf, ctx->last_msg.data(), k);
    buf[k] = 0;
  }
  return ctx->last_code;
}

int ccpt_create(ccpt_ctx** out, int device, const ccpt_options* opts) {
  if (!out) return CCPT_E_INVALID;
  *out = nullptr;
  ccpt_options o;
  if (opts)
    o = *opts;
  else
    ccpt_default_options(&o);
  if (o.mode != CCPT_MODE_CCU && o.mode != CCPT_MODE_CCSN) return CCPT_E_INVALID;
  if (o.upsample < 1 || o.upsample > 1024) return CCPT_E_INVALID;
  if (!(o.window > 0.0 && o.window <= 2.0)) return CCPT_E_INVALID;
  if (o.precision != CCPT_PREC_FP32 && o.precision != CCPT_PREC_BF16X2) return CCPT_E_INVALID;
  if (o.newton_iters < 0 || o.newton_iters > 8) return CCPT_E_INVALID;
  if (!std::isfinite(o.eps)) return CCPT_E_INVALID;
  const int M = (int)std::ceil(o.window * o.upsample - 1e-9);
  if (M < 1 || M > 1536) return CCPT_E_INVALID;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CCPT_E_HIP;
  ccpt_ctx* ctx = new (std::nothrow) ccpt_ctx();
  if (!ctx) return CCPT_E_NOMEM;
  ctx->device = device;
  ctx->o = o;
  ctx->M = M;
  ctx->c = M / 2;
  if (hipSetDevice(device) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->desc_evt, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return CCPT_E_HIP;
  }
  *out = ctx;
  return CCPT_OK;
}

void ccpt_destroy(ccpt_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : ctx->tables) {
    (void)hipFree(kv.second.tw);
    (void)hipFree(kv.second.ky);
    (void)hipFree(kv.second.wb);
  }
  for (auto& r : ctx->refs) {
    (void)hipFree(r.spec);
    (void)hipFree(r.img);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_desc) (void)hipFree(ctx->d_desc);
  if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
  if (ctx->desc_evt) (void)hipEventDestroy(ctx->desc_evt);
  delete ctx;
}

int ccpt_set_reference(ccpt_ctx* ctx, const ccpt_image* refs, int n_refs, void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (!refs || n_refs <= 0) return fail(ctx, CCPT_E_INVALID, "no references given");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n_refs; ++i) {
    rc = check_image(ctx, refs[i].data, refs[i].ny, refs[i].nx, refs[i].pitch, refs[i].dtype,
                     "reference", i);
    if (rc) return rc;
  }
  HIP_CHECK(ctx, hipStreamSynchronize(s));
  // read the references back: the CC-SN domain check and the context's own copy
  std::vector<std::vector<float>> host(n_refs);
  for (int i = 0; i < n_refs; ++i) {
    const ccpt_image& im = refs[i];
    const size_t esz = im.dtype == CCPT_U16 ? 2 : 4;
    std::vector<char> raw((size_t)im.ny * im.pitch * esz);
    HIP_CHECK(ctx, hipMemcpy(raw.data(), im.data, raw.size(), hipMemcpyDeviceToHost));
    host[i].resize((size_t)im.ny * im.nx);
    for (int y = 0; y < im.ny; ++y)
      for (int x = 0; x < im.nx; ++x) {
        const size_t k = (size_t)y * im.pitch + x;
        float v = im.dtype == CCPT_U16 ? (float)((const uint16_t*)raw.data())[k]
                                       : ((const float*)raw.data())[k];
        if (!std::isfinite(v))
          return fail(ctx, CCPT_E_INVALID, "reference %d has a non-finite pixel", i);
        if (ctx->o.mode == CCPT_MODE_CCSN && !(v + ctx->o.eps > 0.0))
          return fail(ctx, CCPT_E_NONPOSITIVE_REF, "reference %d: E + eps <= 0 at (%d, %d)", i,
                      y, x);
        host[i][(size_t)y * im.nx + x] = v;
      }
  }
  // drop the old set (graphs hold pointers to the old spectra through descriptors only)
  HIP_CHECK(ctx, hipDeviceSynchronize());
  for (auto& r : ctx->refs) {
    (void)hipFree(r.spec);
    (void)hipFree(r.img);
  }
  ctx->refs.clear();
  ctx->last_desc.clear();
  size_t tmp_need = 0;
  for (int i = 0; i < n_refs; ++i) {
    const int n = refs[i].nx;
    tmp_need = std::max(tmp_need, (size_t)n * (n / 2 + 1) * sizeof(float2));
    rc = ensure_tables(ctx, n);
    if (rc) return rc;
  }
  float2* T = nullptr;
  HIP_CHECK(ctx, hipMalloc(&T, tmp_need));
  for (int i = 0; i < n_refs; ++i) {
    const int n = refs[i].nx;
    Ref r;
    r.n = n;
    if (hipMalloc(&r.spec, (size_t)n * (n / 2 + 1) * sizeof(float2)) != hipSuccess ||
        hipMalloc(&r.img, (size_t)n * n * sizeof(float)) != hipSuccess) {
      (void)hipFree(T);
      return fail(ctx, CCPT_E_NOMEM, "reference spectra");
    }
    HIP_CHECK(ctx, hipMemcpy(r.img, host[i].data(), (size_t)n * n * sizeof(float),
                             hipMemcpyHostToDevice));
    const int weight = ctx->o.mode == CCPT_MODE_CCSN ? 1 : 0;
    if (launch_spectrum(n, r.img, CCPT_F32, n, 0, 1, weight, (float)ctx->o.eps, 1, T, r.spec,
                        ctx->tables[n].tw, s)) {
      (void)hipFree(T);
      return fail(ctx, CCPT_E_HIP, "reference spectrum launch failed");
    }
    ctx->refs.push_back(r);
  }
  HIP_CHECK(ctx, hipStreamSynchronize(s));
  HIP_CHECK(ctx, hipFree(T));
  return CCPT_OK;
}

int ccpt_track_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                     void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 0 || (n > 0 && (!rois || !out))) return fail(ctx, CCPT_E_INVALID, "bad roi array");
  if (n == 0) return CCPT_OK;
  if (ctx->refs.empty()) return fail(ctx, CCPT_E_NOREF, "no reference set");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < n; ++i) {
    const ccpt_roi& r = rois[i];
    rc = check_image(ctx, r.data, r.ny, r.nx, r.pitch, r.dtype, "roi", i);
    if (rc) return rc;
    if (r.ref_id < 0 || r.ref_id >= (int)ctx->refs.size())
      return fail(ctx, CCPT_E_NOREF, "roi %d: reference id %d not set", i, r.ref_id);
    if (ctx->refs[r.ref_id].n != r.nx)
      return fail(ctx, CCPT_E_INVALID, "roi %d: size %d differs from reference %d (%d)", i, r.nx,
                  r.ref_id, ctx->refs[r.ref_id].n);
  }
  // group by size, largest first (they take longest)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return rois[a].nx > rois[b].nx; });
  std::vector<FrameDesc> desc(n);
  std::vector<int> sig;
  size_t ws_need = 0;
  for (int k = 0; k < n; ++k) {
    const ccpt_roi& r = rois[order[k]];
    FrameDesc d;
    d.data = r.data;
    d.rspec = ctx->refs[r.ref_id].spec;
    d.pitch = r.pitch;
    d.dtype = r.dtype;
    d.out_idx = order[k];
    d.pad = 0;
    desc[k] = d;
    if (sig.empty() || sig[sig.size() - 2] != r.nx) {
      sig.push_back(r.nx);
      sig.push_back(0);
    }
    sig.back()++;
  }
  for (size_t gi = 0; gi < sig.size(); gi += 2) {
    const int nn = sig[gi], cnt = sig[gi + 1];
    const int chunk = std::min(cnt, chunk_for(ctx, nn));
    ws_need = std::max(ws_need, frame_ws_bytes(nn) * (size_t)chunk + 256);
  }
  rc = ensure_ws(ctx, ws_need);
  if (rc) return rc;
  // descriptor upload (skipped when identical to the previous call)
  const size_t bytes = (size_t)n * sizeof(FrameDesc);
  if ((size_t)n > ctx->desc_cap) {
    HIP_CHECK(ctx, hipDeviceSynchronize());
    drop_graphs(ctx);
    if (ctx->d_desc) (void)hipFree(ctx->d_desc);
    if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
    ctx->d_desc = nullptr;
    ctx->h_desc = nullptr;
    size_t cap = std::max<size_t>(n, 64);
    if (hipMalloc(&ctx->d_desc, cap * sizeof(FrameDesc)) != hipSuccess ||
        hipHostMalloc(&ctx->h_desc, cap * sizeof(FrameDesc), hipHostMallocDefault) != hipSuccess) {
      ctx->desc_cap = 0;
      return fail(ctx, CCPT_E_NOMEM, "descriptor table");
    }
    ctx->desc_cap = cap;
    ctx->last_desc.clear();
  }
  const bool same = ctx->last_desc.size() == (size_t)n &&
                    memcmp(ctx->last_desc.data(), desc.data(), bytes) == 0;
  if (!same) {
    HIP_CHECK(ctx, hipEventSynchronize(ctx->desc_evt));
    memcpy(ctx->h_desc, desc.data(), bytes);
    HIP_CHECK(ctx, hipMemcpyAsync(ctx->d_desc, ctx->h_desc, bytes, hipMemcpyHostToDevice, s));
    HIP_CHECK(ctx, hipEventRecord(ctx->desc_evt, s));
    ctx->last_desc = desc;
  }

  auto launch_all = [&]() -> int {
    int first = 0;
    for (size_t gi = 0; gi < sig.size(); gi += 2) {
      const int nn = sig[gi], cnt = sig[gi + 1];
      int r2 = run_group(ctx, nn, ctx->d_desc, first, cnt, out, s);
      if (r2) return r2;
      first += cnt;
    }
    return CCPT_OK;
  };

  const bool use_graph = (ctx->o.flags & CCPT_FLAG_GRAPH) && s != nullptr;
  if (!use_graph) return launch_all();
  GraphKey key{sig, out, s};
  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    hipGraph_t graph;
    HIP_CHECK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int r2 = launch_all();
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (r2) return r2;
    if (e != hipSuccess) return fail(ctx, CCPT_E_HIP, "capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(ctx, CCPT_E_HIP, "instantiate: %s", hipGetErrorString(e));
    it = ctx->graphs.emplace(key, exec).first;
  }
  HIP_CHECK(ctx, hipGraphLaunch(it->second, s));
  return CCPT_OK;
}

int ccpt_track_grad(ccpt_ctx* ctx, const ccpt_roi*, int, const ccpt_result*, const double*,
                    const double*, float*, float*, void*) {
  if (!ctx) return CCPT_E_INVALID;
  return fail(ctx, CCPT_E_UNSUPPORTED, "gradient not built yet");
}

int ccpt_fisher(ccpt_ctx* ctx, const ccpt_image*, double*, void*) {
  if (!ctx) return CCPT_E_INVALID;
  return fail(ctx, CCPT_E_UNSUPPORTED, "fisher not built yet");
}

int ccpt_autotune(ccpt_ctx* ctx, int, int, void*) {
  if (!ctx) return CCPT_E_INVALID;
  return CCPT_OK;
}

}  // extern "C"
