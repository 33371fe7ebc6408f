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

// Shape codes.  A square N x N frame has code N.  A rectangle has code
// kRectCode | trans | NY << 11 | NX, NY x NX being its tall kernel shape
// (one of CCPT_FOR_RECT); trans is set when the frame itself is wide (NX rows
// of NY pixels), which the kernels read transposed.  Tables are shared by
// both orientations (key without the trans bit).
constexpr int kRectCode = 1 << 24;
constexpr int kTransBit = 1 << 23;
bool is_rect(int code) { return (code & kRectCode) != 0; }
int code_ny(int code) { return is_rect(code) ? (code >> 11) & 2047 : code; }
int code_nx(int code) { return is_rect(code) ? code & 2047 : code; }
int code_trans(int code) { return is_rect(code) && (code & kTransBit) ? 1 : 0; }
int table_key(int code) { return code & ~kTransBit; }

// The code of an ny x nx frame, 0 if the shape is not supported.
int shape_code(int ny, int nx) {
  if (ny == nx) return supported_size(ny) ? ny : 0;
  const int a = std::max(ny, nx), b = std::min(ny, nx);
  bool ok = false;
#define CASE(p, q) \
  if (a == p && b == q) ok = true;
  CCPT_FOR_RECT(CASE)
#undef CASE
  if (!ok) return 0;
  return kRectCode | (ny < nx ? kTransBit : 0) | (a << 11) | b;
}

struct SizeTables {
  float2* tw = nullptr;  // N
  void* ky = nullptr;
  void* wb = nullptr;
  unsigned* kfold = nullptr;  // split precision, N >= kWideMinN
  int Mp = 0;
  // FP64 mode
  double2* tw64 = nullptr;  // N
  double2* ky64 = nullptr;  // [Mp][N]
  double2* wb64 = nullptr;  // [N/2+1][Mp]
};

struct Ref {
  int n = 0;                  // shape code
  float2* spec = nullptr;     // conj F[B], N x (N/2+1) (the adjoint always uses it)
  double2* spec64 = nullptr;  // the same in FP64 (FP64 mode)
  float* img = nullptr;       // E as float (N x N), kept for the CC-SN chain rule
  float2* espec = nullptr;    // CC-SN: F[E], N x (N/2+1), for real-time updates
};

// Launch plan of one frame shape (ccpt_plan): chunk size and block plans.
struct Schedule {
  int chunk = 0;          // frames per launch chunk (0 = default)
  int split_blocks = -1;  // FP32: split Stage A below this many row tiles per launch (-1: default)
  int fused_min = -1;     // 256x256: one-kernel correlation from this many frames (-1: default)
};

// Size groups of one call run concurrently on up to kMaxLanes streams.
constexpr int kMaxLanes = 4;

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
  // profiling: events bracketing each launch
  struct Span {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Span> spans;
  std::vector<hipEvent_t> ev_pool;
  hipStream_t cur_stream = nullptr;
  hipEvent_t open_ev = nullptr;
  // adjoint: packed-gradient offsets + accumulator pointers, accumulators
  void* gsmall = nullptr;
  size_t gsmall_cap = 0;
  char* h_small = nullptr;
  size_t h_small_cap = 0;
  hipEvent_t small_evt = nullptr;
  void* acc_buf = nullptr;
  size_t acc_cap = 0;
  // FP32 split-K partials of small launches
  void* ypart = nullptr;
  size_t ypart_cap = 0;
  // per-frame states of a chunk: kept in the initial state between chunks by
  // the Newton kernel; re-initialised after a failed launch
  FrameState* st_buf = nullptr;
  size_t st_cap = 0;
  bool st_dirty = true;
  // partial Newton models of small launches
  void* nparts = nullptr;
  size_t nparts_cap = 0;
  // chunk slots: a group of several chunks runs them alternately on the
  // caller's stream and `aux`, each slot with its own part of the workspace,
  // frame states, split-K and Newton partials (strides below, per slot)
  hipStream_t aux = nullptr;
  hipEvent_t fork_evt = nullptr, join_evt = nullptr;
  size_t slot_ws = 0, slot_st = 0, slot_ypart = 0;
  // concurrent size groups: lane 0 is the caller's stream, lanes 1.. these
  // context-owned streams (default priority), forked from and joined back
  // into the caller's stream by events; each lane has its own workspace,
  // frame states, split-K and Newton partials
  hipStream_t lane_s[kMaxLanes - 1] = {};
  hipEvent_t lane_evt[kMaxLanes - 1] = {};
  int lanes = 0;  // most lanes a call uses (0: kMaxLanes)
  // real-time updates: scratch spectra T and F
  void* rt_buf = nullptr;
  size_t rt_cap = 0;
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

bool fp64(const ccpt_ctx* ctx) { return ctx->o.precision == CCPT_PREC_FP64; }
bool split(const ccpt_ctx* ctx) {
  return ctx->o.precision == CCPT_PREC_BF16X2 || ctx->o.precision == CCPT_PREC_FP16X2;
}

// Longest Newton step before the result falls back to the grid estimate.
// An FP64 grid locates the maximum to a grid step, so a longer step means
// Newton and grid disagree.  FP32 and split-precision grids do not: where
// the correlation is flat near its maximum relative to its size (broad
// spots, the large constant term of CC-SN, large u) neighbouring grid values
// differ by less than their rounding, and the grid maximum can sit tenths of
// a pixel from the true one; their steps are bounded by the half window
// only (the Hessian test and the window test still apply).
double step_limit(const ccpt_ctx* ctx) {
  const double grid = 1.0 / ctx->o.upsample;
  return fp64(ctx) ? grid : std::max(grid, 0.5 * ctx->o.window);
}

template <typename T>
int upload(ccpt_ctx* ctx, T*& dst, const std::vector<T>& src) {
  HIP_CHECK(ctx, hipMalloc(&dst, src.size() * sizeof(T)));
  HIP_CHECK(ctx, hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return CCPT_OK;
}

int ensure_tables(ccpt_ctx* ctx, int code) {
  const int key = table_key(code);
  if (ctx->tables.count(key)) return CCPT_OK;
  const int n = code_ny(code), nx = code_nx(code);
  SizeTables t;
  // the FP64 mode keeps the FP32 tables too (twiddles of the adjoint and Fisher paths)
  HostTables h = build_tables(n, nx, ctx->o.upsample, ctx->M, ctx->c,
                              fp64(ctx) ? CCPT_PREC_FP32 : ctx->o.precision);
  t.Mp = h.Mp;
  HIP_CHECK(ctx, hipMalloc(&t.tw, h.tw.size() * sizeof(float2)));
  HIP_CHECK(ctx, hipMemcpy(t.tw, h.tw.data(), h.tw.size() * sizeof(float2), hipMemcpyHostToDevice));
  HIP_CHECK(ctx, hipMalloc(&t.ky, h.ky.size()));
  HIP_CHECK(ctx, hipMemcpy(t.ky, h.ky.data(), h.ky.size(), hipMemcpyHostToDevice));
  HIP_CHECK(ctx, hipMalloc(&t.wb, h.wb.size()));
  HIP_CHECK(ctx, hipMemcpy(t.wb, h.wb.data(), h.wb.size(), hipMemcpyHostToDevice));
  if (fp64(ctx)) {
    HostTables64 h64 = build_tables64(n, ctx->o.upsample, ctx->M, ctx->c, t.Mp);
    int rc = upload(ctx, t.tw64, h64.tw);
    if (!rc) rc = upload(ctx, t.ky64, h64.ky);
    if (!rc) rc = upload(ctx, t.wb64, h64.wb);
    if (rc) return rc;
  }
  if (split(ctx) && nx >= kWideMinN) {
    const size_t words = (size_t)n * 2 * kfold_rows(t.Mp) * xb_pitch(n);
    if (hipMalloc(&t.kfold, words * sizeof(unsigned)) != hipSuccess)
      return fail(ctx, CCPT_E_NOMEM, "folded table of %zu bytes", words * sizeof(unsigned));
    if (launch_build_kfold(t.kfold, n, ctx->o.upsample, ctx->M, ctx->c, kfold_rows(t.Mp),
                           ctx->o.precision == CCPT_PREC_FP16X2 ? 1 : 0, nullptr))
      return fail(ctx, CCPT_E_HIP, "folded table launch failed");
    HIP_CHECK(ctx, hipDeviceSynchronize());
  }
  ctx->tables[key] = t;
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

// Half-spectrum elements and split-precision words of one frame (shape code).
size_t spec_elems(int code) { return (size_t)code_ny(code) * (code_nx(code) / 2 + 1); }

size_t split_words(int code) { return (size_t)2 * (code_nx(code) / 2) * xb_pitch(code_ny(code)); }

size_t frame_ws_bytes(int n, int precision) {
  if (precision == CCPT_PREC_FP64)
    return 2 * spec_elems(n) * sizeof(double2) + (size_t)(n / row_block64(n)) * sizeof(PeakCand);
  size_t b = 2 * spec_elems(n) * sizeof(float2);
  if (precision == CCPT_PREC_BF16X2 || precision == CCPT_PREC_FP16X2)
    b += split_words(n) * sizeof(unsigned) + (size_t)code_ny(n) * sizeof(float2);  // Xb, Zc
  return b;
}

int default_chunk(int n, int precision) {
  // keep the chunk's spectra well inside the 256 MB Infinity Cache
  const size_t budget = (size_t)192 << 20;
  int c = (int)(budget / frame_ws_bytes(n, precision));
  return std::max(1, std::min(c, 4096));
}

int chunk_for(const ccpt_ctx* ctx, int n) {
  auto it = ctx->sched.find(n);
  if (it != ctx->sched.end() && it->second.chunk > 0) return it->second.chunk;
  return default_chunk(n, ctx->o.precision);
}

int split_blocks_for(const ccpt_ctx* ctx, int n) {
  auto it = ctx->sched.find(n);
  if (it != ctx->sched.end() && it->second.split_blocks >= 0) return it->second.split_blocks;
  return kSplitMaxBlocks;
}

int fused_min_for(const ccpt_ctx* ctx, int n) {
  // the fp16 split takes its operands from the one-kernel correlation only
  if (ctx->o.precision == CCPT_PREC_FP16X2) return 1;
  auto it = ctx->sched.find(n);
  if (it != ctx->sched.end() && it->second.fused_min >= 0) return it->second.fused_min;
  return kFusedMinFrames;
}

// Device memory the launches of one call work in: the context's buffers
// (ccpt_track_batch) or the library's static scratch (ccpt_track_batch_static).
struct CallMem {
  char* ws = nullptr;          // chunk workspace, slot_ws bytes per slot
  size_t slot_ws = 0;
  FrameState* st = nullptr;    // frame states, slot_st entries per slot
  size_t slot_st = 0;
  void* ypart = nullptr;       // FP32 split-K partials, slot_ypart bytes per slot (or none)
  size_t slot_ypart = 0;
  void* nparts = nullptr;      // Newton partial models per slot (or none)
  size_t chunk_bytes = 0;      // > 0: chunks limited to this much workspace
  bool slots = true;           // two chunk slots allowed (CCPT_FLAG_STREAMS)
  bool mark = true;            // profiling events allowed
  bool* st_dirty = nullptr;    // set while a chunk's states may be left non-initial
};

CallMem ctx_mem(ccpt_ctx* ctx) {
  CallMem m;
  m.ws = ctx->ws;
  m.slot_ws = ctx->slot_ws;
  m.st = ctx->st_buf;
  m.slot_st = ctx->slot_st;
  m.ypart = ctx->ypart;
  m.slot_ypart = ctx->slot_ypart;
  m.nparts = ctx->nparts;
  m.st_dirty = &ctx->st_dirty;
  return m;
}

// Carves the workspace for a chunk of `chunk` frames of size n (every part
// 16-byte aligned: spectra rows hold an even number of float2).
void carve(ccpt_ctx* ctx, const CallMem& mem, int n, int chunk, int slot, GroupParams& g) {
  const size_t spec = spec_elems(n);
  char* ws = mem.ws + slot * mem.slot_ws;
  g.st = mem.st + slot * mem.slot_st;
  if (fp64(ctx)) {
    g.T = g.X = nullptr;
    g.Xb = nullptr;
    g.T64 = (double2*)ws;
    g.X64 = g.T64 + spec * chunk;
    g.cand = (PeakCand*)(g.X64 + spec * chunk);
    return;
  }
  g.T = (float2*)ws;
  g.X = g.T + spec * chunk;
  char* p = (char*)(g.X + spec * chunk);
  g.Xb = nullptr;
  g.Zc = nullptr;
  if (split(ctx)) {
    g.Xb = (unsigned*)p;
    p += split_words(n) * sizeof(unsigned) * chunk;
    g.Zc = (float2*)p;
    p += (size_t)code_ny(n) * sizeof(float2) * chunk;
  }
  (void)p;
}

int check_image(ccpt_ctx* ctx, const void* data, int ny, int nx, int pitch, int dtype,
                const char* what, int idx) {
  if (!data) return fail(ctx, CCPT_E_INVALID, "%s %d: null data", what, idx);
  if (dtype != CCPT_U16 && dtype != CCPT_F32 && dtype != CCPT_F64)
    return fail(ctx, CCPT_E_INVALID, "%s %d: unknown dtype %d", what, idx, dtype);
  if (ny <= 0 || nx <= 0 || pitch < nx)
    return fail(ctx, CCPT_E_INVALID, "%s %d: bad shape %dx%d pitch %d", what, idx, ny, nx, pitch);
  if (!shape_code(ny, nx))
    return fail(ctx, CCPT_E_UNSUPPORTED, "%s %d: %dx%d is not a supported shape", what, idx, ny,
                nx);
  const size_t align = dtype_bytes(dtype);
  if ((uintptr_t)data % align)
    return fail(ctx, CCPT_E_INVALID, "%s %d: misaligned data", what, idx);
  return CCPT_OK;
}

// One pixel of a host copy of an image.
double pixel(const void* raw, int dtype, size_t k) {
  if (dtype == CCPT_U16) return (double)((const uint16_t*)raw)[k];
  if (dtype == CCPT_F64) return ((const double*)raw)[k];
  return (double)((const float*)raw)[k];
}

// Calls that work on square frames only (the adjoint, the Fisher information
// and the reference updates).
int require_square(ccpt_ctx* ctx, int ny, int nx, const char* what) {
  if (ny != nx)
    return fail(ctx, CCPT_E_UNSUPPORTED, "%s: %dx%d frames are tracked, but this call takes square "
                "frames only", what, ny, nx);
  return CCPT_OK;
}

GroupParams base_params(ccpt_ctx* ctx, int n) {
  GroupParams g{};
  g.tw = ctx->tables[table_key(n)].tw;
  g.mode = ctx->o.mode;
  g.eps = (float)ctx->o.eps;
  g.eps64 = ctx->o.eps;
  g.tw64 = ctx->tables[table_key(n)].tw64;
  g.trans = code_trans(n);
  g.u = ctx->o.upsample;
  g.M = ctx->M;
  g.c = ctx->c;
  g.newton_iters = ctx->o.newton_iters;
  g.half_window = 0.5 * ctx->o.window;
  g.fused_min = fused_min_for(ctx, n);
  return g;
}

hipEvent_t pool_event(ccpt_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void mark_cb(void* user, int stage, int begin) {
  ccpt_ctx* ctx = (ccpt_ctx*)user;
  hipEvent_t e = pool_event(ctx);
  if (!e) return;
  (void)hipEventRecord(e, ctx->cur_stream);
  if (begin) {
    ctx->open_ev = e;
  } else if (ctx->open_ev) {
    ctx->spans.push_back({stage, ctx->open_ev, e});
    ctx->open_ev = nullptr;
  }
}

Marker marker_of(ccpt_ctx* ctx, hipStream_t s) {
  Marker m;
  if (ctx->o.flags & CCPT_FLAG_PROFILE) {
    ctx->cur_stream = s;
    m.fn = mark_cb;
    m.user = ctx;
  }
  return m;
}

// Bytes of FP32 split-K partials a launch of `count` frames of size n uses
// (0 when the launch is large enough to fill the GPU without splitting).
size_t split_partials_bytes(const ccpt_ctx* ctx, int n, int count) {
  if (ctx->o.precision != CCPT_PREC_FP32) return 0;
  auto it = ctx->tables.find(table_key(n));
  if (it == ctx->tables.end()) return 0;
  const int mtiles = it->second.Mp / 32;
  if ((long)count * mtiles >= split_blocks_for(ctx, n)) return 0;
  return (size_t)count * mtiles * kSplitSlices * 32 * stage_b_k(code_nx(n)) * sizeof(float);
}

// With CCPT_FLAG_STREAMS the chunks of one group run on two streams (not
// when launches are being timed, which needs them in sequence).
bool use_slots(const ccpt_ctx* ctx) {
  return ctx->aux != nullptr && (ctx->o.flags & CCPT_FLAG_STREAMS) &&
         !(ctx->o.flags & CCPT_FLAG_PROFILE);
}

// Launches the whole tracking sequence for one size group, chunk by chunk.
// Frames first..first+count-1 of a plan are uint16 or float32 with an even
// pitch and pixel pairs aligned to their size.
bool pairs_ok(const std::vector<FrameDesc>& desc, int first, int count) {
  for (int i = first; i < first + count; ++i) {
    const FrameDesc& d = desc[i];
    if ((d.dtype != CCPT_U16 && d.dtype != CCPT_F32) || (d.pitch & 1) ||
        ((uintptr_t)d.data & (uintptr_t)(2 * dtype_bytes(d.dtype) - 1)))
      return false;
  }
  return true;
}

int run_group(ccpt_ctx* ctx, const CallMem& mem, int n, const FrameDesc* d_desc, int first,
              int count, ccpt_result* out, hipStream_t s, bool pairs) {
  int chunk = std::min(count, chunk_for(ctx, n));
  if (mem.chunk_bytes) {
    chunk = std::min<int>(chunk, (int)(mem.chunk_bytes / frame_ws_bytes(n, ctx->o.precision)));
    chunk = std::min<int>(chunk, (int)mem.slot_st);
  }
  if (chunk < 1) return fail(ctx, CCPT_E_INVALID, "no workspace for one frame");
  SizeTables& t = ctx->tables[table_key(n)];
  const int ny = code_ny(n), nx = code_nx(n);
  UpdftTables ut{t.ky, t.wb, t.Mp, ctx->o.precision, t.kfold};
  const Marker mark = mem.mark ? marker_of(ctx, s) : Marker{};
  // several chunks: alternate between the two slots (streams s and aux),
  // forked from and joined back into s
  const bool two = count > chunk && mem.slots && use_slots(ctx);
  if (two) {
    HIP_CHECK(ctx, hipEventRecord(ctx->fork_evt, s));
    HIP_CHECK(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_evt, 0));
  }
  // a failed launch leaves no work of this call running on the second stream
  auto failed = [&](const char* what) {
    if (two) (void)hipStreamSynchronize(ctx->aux);
    return fail(ctx, CCPT_E_HIP, "%s launch failed", what);
  };
  for (int c0 = 0, ci = 0; c0 < count; c0 += chunk, ++ci) {
    const int slot = two ? (ci & 1) : 0;
    hipStream_t cs = slot ? ctx->aux : s;
    GroupParams g = base_params(ctx, n);
    g.pairs_ok = pairs ? 1 : 0;
    g.desc = d_desc;
    g.first = first + c0;
    g.count = std::min(chunk, count - c0);
    g.out = out;
    carve(ctx, mem, n, chunk, slot, g);
    // the one-kernel correlation leaves the split for the matrix DFT to make
    if (g.Xb && xcorr_fused(ny, nx, pairs, g.count, g.fused_min)) g.Xb = nullptr;
    if (g.Xb) g.Zc = nullptr;
    const size_t yb = split_partials_bytes(ctx, n, g.count);
    g.ypart = (yb && mem.ypart && yb <= mem.slot_ypart)
                  ? (float*)((char*)mem.ypart + slot * mem.slot_ypart)
                  : nullptr;
    g.nparts = mem.nparts ? (double*)mem.nparts +
                                (size_t)slot * kNewtonSplitMax * kNewtonParts * kNewtonCoef
                          : nullptr;
    if (mem.st_dirty) *mem.st_dirty = true;  // until this chunk's Newton launch has gone in
    if ((fp64(ctx) ? launch_xcorr64(n, g, cs, mark) : launch_xcorr(ny, nx, g, cs, mark)))
      return failed("correlation");
    mark(CCPT_STAGE_UPDFT, 1);
    if ((fp64(ctx) ? launch_updft64(n, g, t.ky64, t.wb64, t.Mp, cs)
                   : launch_updft(ny, nx, g, ut, cs)))
      return failed("upsampled DFT");
    mark(CCPT_STAGE_UPDFT, 0);
    mark(CCPT_STAGE_NEWTON, 1);
    if (launch_newton(ny, nx, g, step_limit(ctx), cs))
      return failed("Newton");
    mark(CCPT_STAGE_NEWTON, 0);
    if (mem.st_dirty) *mem.st_dirty = false;
  }
  if (two) {
    HIP_CHECK(ctx, hipEventRecord(ctx->join_evt, ctx->aux));
    HIP_CHECK(ctx, hipStreamWaitEvent(s, ctx->join_evt, 0));
  }
  return CCPT_OK;
}


// Validated, size-grouped descriptors of a roi array.
struct Plan {
  std::vector<FrameDesc> desc;  // grouped by shape, largest first
  std::vector<int> sig;         // (shape code, count) pairs of the groups
};

// fp32_spec: point the descriptors at the FP32 reference spectra whatever
// the precision (the adjoint works in FP32).
int plan_rois(ccpt_ctx* ctx, const ccpt_roi* rois, int n, Plan& plan, bool fp32_spec = false) {
  if (ctx->refs.empty()) return fail(ctx, CCPT_E_NOREF, "no reference set");
  std::vector<int> code(n);
  for (int i = 0; i < n; ++i) {
    const ccpt_roi& r = rois[i];
    int rc = check_image(ctx, r.data, r.ny, r.nx, r.pitch, r.dtype, "roi", i);
    if (rc) return rc;
    if (r.ref_id < 0 || r.ref_id >= (int)ctx->refs.size())
      return fail(ctx, CCPT_E_NOREF, "roi %d: reference id %d not set", i, r.ref_id);
    code[i] = shape_code(r.ny, r.nx);
    if (ctx->refs[r.ref_id].n != code[i])
      return fail(ctx, CCPT_E_INVALID, "roi %d: shape %dx%d differs from reference %d", i, r.ny,
                  r.nx, r.ref_id);
  }
  // group by shape, largest first (they take longest); stable within a shape
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const long pa = (long)rois[a].ny * rois[a].nx, pb = (long)rois[b].ny * rois[b].nx;
    return pa != pb ? pa > pb : code[a] > code[b];
  });
  plan.desc.resize(n);
  plan.sig.clear();
  for (int k = 0; k < n; ++k) {
    const ccpt_roi& r = rois[order[k]];
    FrameDesc d;
    d.data = r.data;
    const Ref& ref = ctx->refs[r.ref_id];
    d.rspec = (fp64(ctx) && !fp32_spec) ? (const void*)ref.spec64 : (const void*)ref.spec;
    d.pitch = r.pitch;
    d.dtype = r.dtype;
    d.out_idx = order[k];
    d.ref_id = r.ref_id;
    plan.desc[k] = d;
    if (plan.sig.empty() || plan.sig[plan.sig.size() - 2] != code[order[k]]) {
      plan.sig.push_back(code[order[k]]);
      plan.sig.push_back(0);
    }
    plan.sig.back()++;
  }
  // the fp16 split runs the one-kernel correlation only, which reads pixel pairs
  if (ctx->o.precision == CCPT_PREC_FP16X2 && !fp32_spec && !pairs_ok(plan.desc, 0, n))
    return fail(ctx, CCPT_E_UNSUPPORTED,
                "the fp16 split takes uint16 or float32 frames with an even pitch and aligned pairs");
  return CCPT_OK;
}

// Copies the descriptors to the context's device table through a pinned
// staging buffer; skipped when identical to the previous upload.
int upload_desc(ccpt_ctx* ctx, const std::vector<FrameDesc>& desc, hipStream_t s) {
  const size_t n = desc.size();
  const size_t bytes = n * sizeof(FrameDesc);
  if (n > ctx->desc_cap) {
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
  const bool same = ctx->last_desc.size() == n &&
                    memcmp(ctx->last_desc.data(), desc.data(), bytes) == 0;
  if (!same) {
    HIP_CHECK(ctx, hipEventSynchronize(ctx->desc_evt));
    memcpy(ctx->h_desc, desc.data(), bytes);
    HIP_CHECK(ctx, hipMemcpyAsync(ctx->d_desc, ctx->h_desc, bytes, hipMemcpyHostToDevice, s));
    HIP_CHECK(ctx, hipEventRecord(ctx->desc_evt, s));
    ctx->last_desc = desc;
  }
  return CCPT_OK;
}

// Device buffer owned by the context, grown on demand.
int ensure_buf(ccpt_ctx* ctx, void*& p, size_t& cap, size_t bytes) {
  if (bytes <= cap) return CCPT_OK;
  if (p) {
    HIP_CHECK(ctx, hipDeviceSynchronize());
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
    return fail(ctx, CCPT_E_NOMEM, "buffer of %zu bytes", bytes);
  }
  cap = bytes;
  return CCPT_OK;
}

// The frame-state buffer for chunks of up to `count` frames, in the initial
// state (a new buffer, or one left dirty by a failed launch, is initialised on
// stream s before any kernel of the call uses it).
int ensure_state(ccpt_ctx* ctx, size_t count, hipStream_t s) {
  if (count > ctx->st_cap) {
    drop_graphs(ctx);
    size_t cap = ctx->st_cap;
    void* p = ctx->st_buf;
    int rc = ensure_buf(ctx, p, cap, count * sizeof(FrameState));
    ctx->st_buf = (FrameState*)p;
    ctx->st_cap = cap / sizeof(FrameState);
    if (rc) return rc;
    ctx->st_dirty = true;
  }
  if (!ctx->nparts) {
    // one share per chunk slot (two) or lane (kMaxLanes)
    const size_t bytes =
        (size_t)kMaxLanes * kNewtonSplitMax * kNewtonParts * kNewtonCoef * sizeof(double);
    int rc = ensure_buf(ctx, ctx->nparts, ctx->nparts_cap, bytes);
    if (rc) return rc;
  }
  if (ctx->st_dirty) {
    if (launch_init_state(ctx->st_buf, (int)ctx->st_cap, s))
      return fail(ctx, CCPT_E_HIP, "state initialisation launch failed");
    ctx->st_dirty = false;
  }
  return CCPT_OK;
}

// The streams and events of lanes 1.. (default priority).
int create_lanes(ccpt_ctx* ctx) {
  static_assert(kMaxLanes >= 2, "the two chunk slots use two Newton partial shares");
  for (int l = 0; l < kMaxLanes - 1; ++l)
    if (hipStreamCreateWithFlags(&ctx->lane_s[l], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->lane_evt[l], hipEventDisableTiming) != hipSuccess)
      return -1;
  return 0;
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
  if (o.precision != CCPT_PREC_FP32 && o.precision != CCPT_PREC_BF16X2 &&
      o.precision != CCPT_PREC_FP16X2 &&
      o.precision != CCPT_PREC_FP64)
    return CCPT_E_INVALID;
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
  if (hipSetDevice(device) != hipSuccess || scratch_setup(device) != 0 ||
      hipEventCreateWithFlags(&ctx->desc_evt, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->fork_evt, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->join_evt, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) != hipSuccess ||
      create_lanes(ctx) != 0 ||
      hipEventCreateWithFlags(&ctx->small_evt, hipEventDisableTiming) != hipSuccess) {
    ccpt_destroy(ctx);
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
  for (auto& sp : ctx->spans) {
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : ctx->tables) {
    (void)hipFree(kv.second.tw);
    (void)hipFree(kv.second.ky);
    (void)hipFree(kv.second.wb);
    if (kv.second.kfold) (void)hipFree(kv.second.kfold);
    if (kv.second.tw64) (void)hipFree(kv.second.tw64);
    if (kv.second.ky64) (void)hipFree(kv.second.ky64);
    if (kv.second.wb64) (void)hipFree(kv.second.wb64);
  }
  for (auto& r : ctx->refs) {
    (void)hipFree(r.spec);
    if (r.spec64) (void)hipFree(r.spec64);
    if (r.espec) (void)hipFree(r.espec);
    (void)hipFree(r.img);
  }
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_desc) (void)hipFree(ctx->d_desc);
  if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
  if (ctx->desc_evt) (void)hipEventDestroy(ctx->desc_evt);
  if (ctx->fork_evt) (void)hipEventDestroy(ctx->fork_evt);
  if (ctx->join_evt) (void)hipEventDestroy(ctx->join_evt);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  for (int l = 0; l < kMaxLanes - 1; ++l) {
    if (ctx->lane_s[l]) (void)hipStreamDestroy(ctx->lane_s[l]);
    if (ctx->lane_evt[l]) (void)hipEventDestroy(ctx->lane_evt[l]);
  }
  if (ctx->small_evt) (void)hipEventDestroy(ctx->small_evt);
  if (ctx->gsmall) (void)hipFree(ctx->gsmall);
  if (ctx->acc_buf) (void)hipFree(ctx->acc_buf);
  if (ctx->ypart) (void)hipFree(ctx->ypart);
  if (ctx->st_buf) (void)hipFree(ctx->st_buf);
  if (ctx->nparts) (void)hipFree(ctx->nparts);
  if (ctx->rt_buf) (void)hipFree(ctx->rt_buf);
  if (ctx->h_small) (void)hipHostFree(ctx->h_small);
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
    if (fp64(ctx) && refs[i].ny != refs[i].nx)
      return fail(ctx, CCPT_E_UNSUPPORTED, "reference %d: the FP64 mode takes square frames only",
                  i);
    if (ctx->o.precision == CCPT_PREC_FP16X2 && !(refs[i].ny == 256 && refs[i].nx == 256))
      return fail(ctx, CCPT_E_UNSUPPORTED, "reference %d: the fp16 split takes 256x256 frames only",
                  i);
  }
  HIP_CHECK(ctx, hipStreamSynchronize(s));
  // read the references back: the CC-SN domain check and the context's own copy
  std::vector<std::vector<double>> host(n_refs);
  for (int i = 0; i < n_refs; ++i) {
    const ccpt_image& im = refs[i];
    std::vector<char> raw(((size_t)(im.ny - 1) * im.pitch + im.nx) * dtype_bytes(im.dtype));
    HIP_CHECK(ctx, hipMemcpy(raw.data(), im.data, raw.size(), hipMemcpyDeviceToHost));
    host[i].resize((size_t)im.ny * im.nx);
    for (int y = 0; y < im.ny; ++y)
      for (int x = 0; x < im.nx; ++x) {
        const double v = pixel(raw.data(), im.dtype, (size_t)y * im.pitch + x);
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
    if (r.spec64) (void)hipFree(r.spec64);
    if (r.espec) (void)hipFree(r.espec);
    (void)hipFree(r.img);
  }
  ctx->refs.clear();
  ctx->last_desc.clear();
  // scratch: one spectrum (FP64 size) plus the FP64 image of the FP64 mode
  size_t tmp_need = 0;
  for (int i = 0; i < n_refs; ++i) {
    const int code = shape_code(refs[i].ny, refs[i].nx);
    tmp_need = std::max(tmp_need, spec_elems(code) * sizeof(double2) +
                                      (size_t)refs[i].ny * refs[i].nx * sizeof(double));
    rc = ensure_tables(ctx, code);
    if (rc) return rc;
  }
  char* tmp = nullptr;
  HIP_CHECK(ctx, hipMalloc(&tmp, tmp_need));
  float2* T = (float2*)tmp;
  for (int i = 0; i < n_refs; ++i) {
    const int n = refs[i].nx;  // (square frames: the size)
    const int code = shape_code(refs[i].ny, refs[i].nx);
    const size_t npx = (size_t)refs[i].ny * refs[i].nx;
    const SizeTables& st = ctx->tables[table_key(code)];
    Ref r;
    r.n = code;
    if (hipMalloc(&r.spec, spec_elems(code) * sizeof(float2)) != hipSuccess ||
        hipMalloc(&r.img, npx * sizeof(float)) != hipSuccess ||
        (fp64(ctx) && hipMalloc(&r.spec64, spec_elems(n) * sizeof(double2)) != hipSuccess)) {
      (void)hipFree(tmp);
      if (r.spec) (void)hipFree(r.spec);
      if (r.img) (void)hipFree(r.img);
      return fail(ctx, CCPT_E_NOMEM, "reference spectra");
    }
    ctx->refs.push_back(r);
    std::vector<float> img32(host[i].begin(), host[i].end());
    HIP_CHECK(ctx, hipMemcpy(r.img, img32.data(), npx * sizeof(float), hipMemcpyHostToDevice));
    const int weight = ctx->o.mode == CCPT_MODE_CCSN ? 1 : 0;
    // the image is stored as given (pitch nx); a wide one is read transposed
    if (launch_spectrum(code_ny(code), code_nx(code), r.img, CCPT_F32, refs[i].nx, 0,
                        code_trans(code), 1, weight, (float)ctx->o.eps, 1, T, r.spec, st.tw, s)) {
      (void)hipFree(tmp);
      return fail(ctx, CCPT_E_HIP, "reference spectrum launch failed");
    }
    if (ctx->o.mode == CCPT_MODE_CCSN) {
      // F[E] itself (held tall), the state of real-time updates (B = -1/(E+eps)
      // is not linear in E)
      Ref& rr = ctx->refs.back();
      if (hipMalloc(&rr.espec, spec_elems(code) * sizeof(float2)) != hipSuccess) {
        (void)hipFree(tmp);
        return fail(ctx, CCPT_E_NOMEM, "reference spectra");
      }
      HIP_CHECK(ctx, hipStreamSynchronize(s));
      if (launch_spectrum(code_ny(code), code_nx(code), r.img, CCPT_F32, refs[i].nx, 0,
                          code_trans(code), 1, 0, 0.f, 0, T, rr.espec, st.tw, s)) {
        (void)hipFree(tmp);
        return fail(ctx, CCPT_E_HIP, "reference spectrum launch failed");
      }
    }
    if (fp64(ctx)) {
      // the FP64 spectrum from the reference's own values, not their FP32 copy
      double2* T64 = (double2*)tmp;
      double* img64 = (double*)(T64 + spec_elems(n));
      HIP_CHECK(ctx, hipStreamSynchronize(s));
      HIP_CHECK(ctx, hipMemcpy(img64, host[i].data(), (size_t)n * n * sizeof(double),
                               hipMemcpyHostToDevice));
      if (launch_spectrum64(n, img64, CCPT_F64, n, 0, 1, weight, ctx->o.eps, 1, T64, r.spec64,
                            ctx->tables[n].tw64, s)) {
        (void)hipFree(tmp);
        return fail(ctx, CCPT_E_HIP, "reference spectrum launch failed");
      }
    }
    HIP_CHECK(ctx, hipStreamSynchronize(s));
  }
  HIP_CHECK(ctx, hipFree(tmp));
  return CCPT_OK;
}

int ccpt_track_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                     void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 0 || (n > 0 && (!rois || !out))) return fail(ctx, CCPT_E_INVALID, "bad roi array");
  if (n == 0) return CCPT_OK;
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Plan plan;
  rc = plan_rois(ctx, rois, n, plan);
  if (rc) return rc;
  const std::vector<int>& sig = plan.sig;
  const int ngroups = (int)sig.size() / 2;
  // size groups on lanes: the most expensive first, each to the lane with the
  // least work so far (work = the group's FFT and matrix-DFT flops); one lane
  // when profiling (stage timing follows one stream)
  const int want = ctx->lanes > 0 ? ctx->lanes : kMaxLanes;
  const int nl = (ctx->o.flags & CCPT_FLAG_PROFILE) ? 1 : std::max(1, std::min(ngroups, want));
  std::vector<int> lane_of(ngroups, 0);
  if (nl > 1) {
    std::vector<double> cost(ngroups), load(nl, 0.0);
    std::vector<int> order(ngroups);
    for (int gi = 0; gi < ngroups; ++gi) {
      const int nn = sig[2 * gi];
      const double ny = code_ny(nn), nx = code_nx(nn), h = nx / 2 + 1, m = ctx->M;
      cost[gi] = sig[2 * gi + 1] * (10.0 * ny * nx * std::log2(ny * nx) + 8.0 * m * ny * h + 4.0 * m * m * h);
      order[gi] = gi;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int gi : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      lane_of[gi] = l;
      load[l] += cost[gi];
    }
  }
  // per-lane needs (one lane: per chunk slot, two slots when some group has
  // several chunks and two-stream chunks are on)
  std::vector<size_t> lws(nl, 0), lst(nl, 0), lyp(nl, 0);
  int nslots = 1;
  for (int gi = 0; gi < ngroups; ++gi) {
    const int nn = sig[2 * gi], cnt = sig[2 * gi + 1], l = lane_of[gi];
    const int chunk = std::min(cnt, chunk_for(ctx, nn));
    lws[l] = std::max(lws[l], frame_ws_bytes(nn, ctx->o.precision) * (size_t)chunk + 256);
    lst[l] = std::max(lst[l], (size_t)chunk);
    lyp[l] = std::max(lyp[l], split_partials_bytes(ctx, nn, chunk));
    lyp[l] = std::max(lyp[l], split_partials_bytes(ctx, nn, cnt % chunk));
    if (nl == 1 && cnt > chunk && use_slots(ctx)) nslots = 2;
  }
  std::vector<size_t> ows(nl + 1, 0), ost(nl + 1, 0), oyp(nl + 1, 0);
  for (int l = 0; l < nl; ++l) {
    lws[l] = (lws[l] + 255) / 256 * 256;
    lyp[l] = (lyp[l] + 255) / 256 * 256;
    ows[l + 1] = ows[l] + lws[l] * nslots;
    ost[l + 1] = ost[l] + lst[l] * nslots;
    oyp[l + 1] = oyp[l] + lyp[l] * nslots;
  }
  rc = ensure_ws(ctx, ows[nl]);
  if (rc) return rc;
  ctx->slot_ws = lws[0];
  rc = ensure_state(ctx, ost[nl], s);
  if (rc) return rc;
  ctx->slot_st = lst[0];
  if (oyp[nl] > ctx->ypart_cap) {
    drop_graphs(ctx);
    rc = ensure_buf(ctx, ctx->ypart, ctx->ypart_cap, oyp[nl]);
    if (rc) return rc;
  }
  ctx->slot_ypart = lyp[0];
  rc = upload_desc(ctx, plan.desc, s);
  if (rc) return rc;

  auto launch_all = [&]() -> int {
    std::vector<int> first(ngroups, 0);
    for (int gi = 1; gi < ngroups; ++gi) first[gi] = first[gi - 1] + sig[2 * gi - 1];
    // lanes 1.. start after everything already queued on the caller's stream
    if (nl > 1) {
      HIP_CHECK(ctx, hipEventRecord(ctx->fork_evt, s));
      for (int l = 1; l < nl; ++l) HIP_CHECK(ctx, hipStreamWaitEvent(ctx->lane_s[l - 1], ctx->fork_evt, 0));
    }
    int r2 = CCPT_OK;
    for (int l = 0; l < nl && r2 == CCPT_OK; ++l) {
      CallMem mem = ctx_mem(ctx);
      mem.ws = ctx->ws + ows[l];
      mem.slot_ws = lws[l];
      mem.st = ctx->st_buf + ost[l];
      mem.slot_st = lst[l];
      mem.ypart = ctx->ypart ? (char*)ctx->ypart + oyp[l] : nullptr;
      mem.slot_ypart = lyp[l];
      mem.nparts = ctx->nparts ? (double*)ctx->nparts +
                                     (size_t)l * kNewtonSplitMax * kNewtonParts * kNewtonCoef
                               : nullptr;
      if (nl > 1) mem.slots = false;
      hipStream_t ls = l ? ctx->lane_s[l - 1] : s;
      for (int gi = 0; gi < ngroups && r2 == CCPT_OK; ++gi) {
        if (lane_of[gi] != l) continue;
        const int nn = sig[2 * gi], cnt = sig[2 * gi + 1];
        r2 = run_group(ctx, mem, nn, ctx->d_desc, first[gi], cnt, out, ls,
                       pairs_ok(plan.desc, first[gi], cnt));
      }
    }
    // every lane that was forked joins back, also after a failed launch
    for (int l = 1; l < nl; ++l) {
      if (hipEventRecord(ctx->lane_evt[l - 1], ctx->lane_s[l - 1]) != hipSuccess ||
          hipStreamWaitEvent(s, ctx->lane_evt[l - 1], 0) != hipSuccess) {
        (void)hipStreamSynchronize(ctx->lane_s[l - 1]);
        if (r2 == CCPT_OK) r2 = fail(ctx, CCPT_E_HIP, "joining lane %d failed", l);
      }
    }
    return r2;
  };

  const bool use_graph = (ctx->o.flags & CCPT_FLAG_GRAPH) && !(ctx->o.flags & CCPT_FLAG_PROFILE) &&
                         s != nullptr;
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

int ccpt_track_batch_static(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                            void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 0 || (n > 0 && (!rois || !out))) return fail(ctx, CCPT_E_INVALID, "bad roi array");
  if (n > CCPT_STATIC_MAX_ROIS)
    return fail(ctx, CCPT_E_INVALID, "%d rois exceed the static scratch's %d", n,
                CCPT_STATIC_MAX_ROIS);
  if (n == 0) return CCPT_OK;
  int rc = set_device(ctx);
  if (rc) return rc;
  char* base = (char*)scratch_ptr(ctx->device);
  if (!base) return fail(ctx, CCPT_E_HIP, "static scratch not set up on device %d", ctx->device);
  hipStream_t s = (hipStream_t)stream;
  Plan plan;
  rc = plan_rois(ctx, rois, n, plan);
  if (rc) return rc;
  // scratch layout: descriptors | frame states of one chunk | chunk workspace
  const size_t desc_bytes = ((size_t)n * sizeof(FrameDesc) + 255) / 256 * 256;
  constexpr size_t kStates = 4096;  // the largest chunk of any schedule
  const size_t st_bytes = (kStates * sizeof(FrameState) + 255) / 256 * 256;
  CallMem mem;
  mem.st = (FrameState*)(base + desc_bytes);
  mem.slot_st = kStates;
  mem.ws = base + desc_bytes + st_bytes;
  mem.chunk_bytes = kScratchBytes - desc_bytes - st_bytes;
  mem.slots = false;
  mem.mark = false;
  for (size_t gi = 0; gi < plan.sig.size(); gi += 2)
    if (frame_ws_bytes(plan.sig[gi], ctx->o.precision) > mem.chunk_bytes)
      return fail(ctx, CCPT_E_INVALID, "one %dx%d frame needs %zu bytes of workspace, more than "
                  "the static scratch holds", code_ny(plan.sig[gi]), code_nx(plan.sig[gi]),
                  frame_ws_bytes(plan.sig[gi], ctx->o.precision));
  FrameDesc* d_desc = (FrameDesc*)base;
  // from pageable memory: the host array is consumed before the call returns
  HIP_CHECK(ctx, hipMemcpyAsync(d_desc, plan.desc.data(), (size_t)n * sizeof(FrameDesc),
                                hipMemcpyHostToDevice, s));
  // whatever an earlier call left in the states: back to the initial state
  if (launch_init_state(mem.st, (int)kStates, s))
    return fail(ctx, CCPT_E_HIP, "state initialisation launch failed");
  int first = 0;
  for (size_t gi = 0; gi < plan.sig.size(); gi += 2) {
    const int nn = plan.sig[gi], cnt = plan.sig[gi + 1];
    rc = run_group(ctx, mem, nn, d_desc, first, cnt, out, s, pairs_ok(plan.desc, first, cnt));
    if (rc) return rc;
    first += cnt;
  }
  return CCPT_OK;
}

int ccpt_track_grad(ccpt_ctx* ctx, const ccpt_roi* rois, int n, const ccpt_result* fwd,
                    const double* g_d, const double* g_peak, float* g_frames, float* g_ref,
                    void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 0 || (n > 0 && (!rois || !fwd || !g_d)))
    return fail(ctx, CCPT_E_INVALID, "bad gradient arguments");
  if (!g_frames && !g_ref) return CCPT_OK;
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    // no rois: every reference gradient is an empty sum
    size_t total = 0;
    for (const Ref& r : ctx->refs) total += (size_t)code_ny(r.n) * code_nx(r.n);
    if (g_ref && total && launch_zero(g_ref, total * sizeof(float), s))
      return fail(ctx, CCPT_E_HIP, "zero launch failed");
    return CCPT_OK;
  }
  for (int i = 0; i < n; ++i) {
    rc = require_square(ctx, rois[i].ny, rois[i].nx, "ccpt_track_grad");
    if (rc) return rc;
  }
  Plan plan;
  rc = plan_rois(ctx, rois, n, plan, true);
  if (rc) return rc;
  const int nrefs = (int)ctx->refs.size();
  // packed offsets of the frame gradients (roi order) and of the reference gradients
  std::vector<long> goff(n);
  long acc_el = 0;
  for (int i = 0; i < n; ++i) {
    goff[i] = acc_el;
    acc_el += (long)rois[i].ny * rois[i].nx;
  }
  std::vector<long> roff(nrefs), aoff(nrefs);
  long ro = 0, ao = 0;
  for (int r = 0; r < nrefs; ++r) {
    const int nn = ctx->refs[r].n;
    roff[r] = ro;
    ro += (long)nn * nn;
    aoff[r] = ao;
    ao += (long)spec_elems(nn);
  }
  // workspace per frame: F[A], QA, QB, T spectra and one image
  auto per_frame = [](int nn) { return 4 * spec_elems(nn) * sizeof(float2) + (size_t)nn * nn * 4; };
  const size_t budget = (size_t)256 << 20;
  size_t ws_need = 0, img_need = 0;
  for (size_t gi = 0; gi < plan.sig.size(); gi += 2) {
    const int nn = plan.sig[gi], cnt = plan.sig[gi + 1];
    const int chunk = std::max(1, std::min<int>(cnt, (int)(budget / per_frame(nn))));
    ws_need = std::max(ws_need, per_frame(nn) * chunk + 256);
  }
  for (int r = 0; r < nrefs; ++r)
    img_need = std::max(img_need, per_frame(ctx->refs[r].n) + 256);
  rc = ensure_ws(ctx, std::max(ws_need, img_need));
  if (rc) return rc;
  const size_t small_bytes = (size_t)n * sizeof(long) + (size_t)nrefs * sizeof(void*);
  rc = ensure_buf(ctx, ctx->gsmall, ctx->gsmall_cap, small_bytes);
  if (rc) return rc;
  if (g_ref) {
    rc = ensure_buf(ctx, ctx->acc_buf, ctx->acc_cap, (size_t)ao * sizeof(float2));
    if (rc) return rc;
  }
  rc = upload_desc(ctx, plan.desc, s);
  if (rc) return rc;
  // small table upload through pinned staging
  HIP_CHECK(ctx, hipEventSynchronize(ctx->small_evt));
  if (small_bytes > ctx->h_small_cap) {
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    ctx->h_small = nullptr;
    ctx->h_small_cap = 0;
    if (hipHostMalloc(&ctx->h_small, small_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(ctx, CCPT_E_NOMEM, "pinned staging");
    ctx->h_small_cap = small_bytes;
  }
  memcpy(ctx->h_small, goff.data(), (size_t)n * sizeof(long));
  float2** accp = (float2**)(ctx->h_small + (size_t)n * sizeof(long));
  for (int r = 0; r < nrefs; ++r)
    accp[r] = g_ref ? (float2*)ctx->acc_buf + aoff[r] : nullptr;
  HIP_CHECK(ctx, hipMemcpyAsync(ctx->gsmall, ctx->h_small, small_bytes, hipMemcpyHostToDevice, s));
  HIP_CHECK(ctx, hipEventRecord(ctx->small_evt, s));
  const long* d_goff = (const long*)ctx->gsmall;
  float2* const* d_acc = (float2* const*)((char*)ctx->gsmall + (size_t)n * sizeof(long));
  if (g_ref && launch_zero(ctx->acc_buf, (size_t)ao * sizeof(float2), s))
    return fail(ctx, CCPT_E_HIP, "zero launch failed");

  const Marker mark = marker_of(ctx, s);
  const int mode = ctx->o.mode;
  const float eps = (float)ctx->o.eps;
  int first = 0;
  mark(CCPT_STAGE_GRAD, 1);
  for (size_t gi = 0; gi < plan.sig.size(); gi += 2) {
    const int nn = plan.sig[gi], cnt = plan.sig[gi + 1];
    const int chunk = std::max(1, std::min<int>(cnt, (int)(budget / per_frame(nn))));
    const float2* tw = ctx->tables[nn].tw;
    const size_t spec = spec_elems(nn);
    for (int c0 = 0; c0 < cnt; c0 += chunk) {
      const int count = std::min(chunk, cnt - c0);
      float2* T = (float2*)ctx->ws;
      float2* FA = T + spec * chunk;
      float2* QA = FA + spec * chunk;
      float2* QB = QA + spec * chunk;
      float* img = (float*)(QB + spec * chunk);
      const int f0 = first + c0;
      if (launch_frame_spectra(nn, nn, 0, ctx->d_desc, f0, count, mode, eps, T, FA, tw, s) ||
          launch_grad_psi(nn, ctx->d_desc, f0, count, fwd, g_d, g_peak, FA, QA,
                          g_ref ? QB : nullptr, s))
        return fail(ctx, CCPT_E_HIP, "gradient launch failed");
      if (g_frames && (launch_inverse(nn, nn, QA, count, 2.0f, T, img, tw, s) ||
                       launch_grad_frames(nn, ctx->d_desc, f0, count, img, d_goff, g_frames, mode,
                                          eps, s)))
        return fail(ctx, CCPT_E_HIP, "frame gradient launch failed");
      if (g_ref && launch_ref_accum(nn, ctx->d_desc, f0, count, QB, d_acc, s))
        return fail(ctx, CCPT_E_HIP, "reference gradient launch failed");
    }
    first += cnt;
  }
  if (g_ref) {
    for (int r = 0; r < nrefs; ++r) {
      const int nn = ctx->refs[r].n;
      float2* T = (float2*)ctx->ws;
      float* img = (float*)(T + spec_elems(nn));
      if (launch_inverse(nn, nn, (float2*)ctx->acc_buf + aoff[r], 1, 2.0f, T, img, ctx->tables[nn].tw,
                         s) ||
          launch_grad_ref_chain(img, ctx->refs[r].img, nn * nn, mode, eps, g_ref + roff[r], s))
        return fail(ctx, CCPT_E_HIP, "reference gradient launch failed");
    }
  }
  mark(CCPT_STAGE_GRAD, 0);
  return CCPT_OK;
}

int ccpt_fisher(ccpt_ctx* ctx, const ccpt_image* mu, double* fisher, void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (!mu || !fisher) return fail(ctx, CCPT_E_INVALID, "null argument");
  int rc = check_image(ctx, mu->data, mu->ny, mu->nx, mu->pitch, mu->dtype, "mean image", 0);
  if (!rc) rc = require_square(ctx, mu->ny, mu->nx, "ccpt_fisher");
  if (rc) return rc;
  rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int n = mu->nx;
  HIP_CHECK(ctx, hipStreamSynchronize(s));
  {
    std::vector<char> raw(((size_t)(mu->ny - 1) * mu->pitch + mu->nx) * dtype_bytes(mu->dtype));
    HIP_CHECK(ctx, hipMemcpy(raw.data(), mu->data, raw.size(), hipMemcpyDeviceToHost));
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double v = pixel(raw.data(), mu->dtype, (size_t)y * mu->pitch + x);
        if (!(v > 0.0) || !std::isfinite(v))
          return fail(ctx, CCPT_E_INVALID, "mean image must be > 0 and finite (%d, %d)", y, x);
      }
  }
  rc = ensure_tables(ctx, n);
  if (rc) return rc;
  const size_t spec = spec_elems(n);
  const int nblocks = 64;
  const size_t bytes = 4 * spec * sizeof(float2) + 2 * (size_t)n * n * sizeof(float) +
                       (size_t)nblocks * 3 * sizeof(double) + 256;
  char* tmp = nullptr;
  HIP_CHECK(ctx, hipMalloc(&tmp, bytes));
  float2* F = (float2*)tmp;
  float2* Dy = F + spec;
  float2* Dx = Dy + spec;
  float2* T = Dx + spec;
  float* iy = (float*)(T + spec);
  float* ix = iy + (size_t)n * n;
  double* part = (double*)(((uintptr_t)(ix + (size_t)n * n) + 15) & ~(uintptr_t)15);
  const float2* tw = ctx->tables[n].tw;
  int bad = launch_spectrum(n, n, mu->data, mu->dtype, mu->pitch, 0, 0, 1, 0, 0.f, 0, T, F, tw,
                            s) ||
            launch_fisher_deriv(n, F, Dy, Dx, s) || launch_inverse(n, n, Dy, 1, 2.0f, T, iy, tw, s) ||
            launch_inverse(n, n, Dx, 1, 2.0f, T, ix, tw, s) ||
            launch_fisher_reduce(iy, ix, mu->data, mu->dtype, mu->pitch, n, part, nblocks, fisher, s);
  hipError_t e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (bad) return fail(ctx, CCPT_E_HIP, "fisher launch failed");
  if (e != hipSuccess) return fail(ctx, CCPT_E_HIP, "fisher: %s", hipGetErrorString(e));
  return CCPT_OK;
}

int ccpt_mean_aligned(ccpt_ctx* ctx, const ccpt_roi* rois, int n, const ccpt_result* fwd,
                      float* out, void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 1 || !rois || !fwd || !out) return fail(ctx, CCPT_E_INVALID, "bad arguments");
  int rc = set_device(ctx);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int N = rois[0].nx;
  std::vector<FrameDesc> desc(n);
  for (int i = 0; i < n; ++i) {
    const ccpt_roi& r = rois[i];
    rc = check_image(ctx, r.data, r.ny, r.nx, r.pitch, r.dtype, "roi", i);
    if (!rc) rc = require_square(ctx, r.ny, r.nx, "ccpt_mean_aligned");
    if (rc) return rc;
    if (r.nx != N) return fail(ctx, CCPT_E_INVALID, "roi %d: size %d differs from %d", i, r.nx, N);
    desc[i] = FrameDesc{r.data, nullptr, r.pitch, r.dtype, i, 0};
  }
  rc = ensure_tables(ctx, N);
  if (rc) return rc;
  const size_t spec = spec_elems(N);
  const size_t per_frame = 2 * spec * sizeof(float2);  // T and the frame's spectrum
  const int chunk = std::max(1, std::min<int>(n, (int)(((size_t)256 << 20) / per_frame)));
  const size_t head = spec * sizeof(float2) + 256;  // accumulator, counter
  rc = ensure_ws(ctx, head + per_frame * chunk);
  if (rc) return rc;
  rc = upload_desc(ctx, desc, s);
  if (rc) return rc;
  float2* acc = (float2*)ctx->ws;
  unsigned* cnt = (unsigned*)(acc + spec);
  float2* T = (float2*)((char*)ctx->ws + head);
  float2* F = T + spec * chunk;
  const float2* tw = ctx->tables[N].tw;
  if (launch_zero(acc, head, s)) return fail(ctx, CCPT_E_HIP, "zero launch failed");
  for (int c0 = 0; c0 < n; c0 += chunk) {
    const int count = std::min(chunk, n - c0);
    if (launch_frame_spectra(N, N, 0, ctx->d_desc, c0, count, CCPT_MODE_CCU, 0.f, T, F, tw, s) ||
        launch_align_accumulate(N, ctx->d_desc, c0, count, fwd, F, acc, cnt, s))
      return fail(ctx, CCPT_E_HIP, "alignment launch failed");
  }
  // the row pass of the inverse returns half the unnormalised transform
  if (launch_inverse(N, N, acc, 1, 2.0f / ((float)N * (float)N), T, out, tw, s) ||
      launch_scale_by_count(out, N * N, 1.0f, cnt, s))
    return fail(ctx, CCPT_E_HIP, "inverse launch failed");
  return CCPT_OK;
}

int ccpt_track_update(ccpt_ctx* ctx, const ccpt_roi* roi, double a0, ccpt_result* out,
                      void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (!roi || !out || !(a0 >= 0.0 && a0 <= 1.0))
    return fail(ctx, CCPT_E_INVALID, "bad arguments");
  if (fp64(ctx)) return fail(ctx, CCPT_E_UNSUPPORTED, "real-time updates need FP32 or BF16X2 precision");
  int rc = ccpt_track_batch(ctx, roi, 1, out, stream);  // validates roi and reference id
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  Ref& R = ctx->refs[roi->ref_id];
  const int code = R.n;
  const int ny = code_ny(code), nx = code_nx(code), tr = code_trans(code);
  const size_t spec = spec_elems(code);
  // scratch: two spectra, and for a rectangle in CC-SN the updated E in the
  // tall layout (the context's copy of a rectangle's E is read by nothing:
  // the adjoint takes square frames only)
  const size_t img_bytes = is_rect(code) ? (size_t)ny * nx * sizeof(float) : 0;
  rc = ensure_buf(ctx, ctx->rt_buf, ctx->rt_cap, 2 * spec * sizeof(float2) + img_bytes);
  if (rc) return rc;
  float2* T = (float2*)ctx->rt_buf;
  float2* F = T + spec;
  float* img = is_rect(code) ? (float*)(F + spec) : R.img;
  const float2* tw = ctx->tables[table_key(code)].tw;
  const float fa0 = (float)a0, fb1 = (float)(1.0 - a0);
  // the frame's own spectrum F[I] (track_batch left its descriptor at index 0)
  if (launch_frame_spectra(ny, nx, tr, ctx->d_desc, 0, 1, CCPT_MODE_CCU, 0.f, T, F, tw, s))
    return fail(ctx, CCPT_E_HIP, "frame spectrum launch failed");
  if (ctx->o.mode == CCPT_MODE_CCU) {
    if (launch_rt_update(ny, nx, tr, out, F, R.spec, fa0, fb1, 1, s))
      return fail(ctx, CCPT_E_HIP, "reference update launch failed");
  } else {
    // update F[E], then E (tall layout), then conj F[-1/(E+eps)]
    if (launch_rt_update(ny, nx, tr, out, F, R.espec, fa0, fb1, 0, s) ||
        launch_inverse(ny, nx, R.espec, 1, 2.0f / ((float)ny * (float)nx), T, img, tw, s) ||
        launch_spectrum(ny, nx, img, CCPT_F32, nx, 0, 0, 1, 1, (float)ctx->o.eps, 1, T, R.spec, tw,
                        s))
      return fail(ctx, CCPT_E_HIP, "reference update launch failed");
  }
  return CCPT_OK;
}

int ccpt_drift_filter(const double* r, int n, double a0, double rate_limit, double* state,
                      double* out) {
  if (n < 0 || (n > 0 && (!r || !out)) || !state || !(a0 >= 0.0 && a0 <= 1.0) ||
      !(rate_limit >= 0.0) || !(state[2] >= 0.0))
    return CCPT_E_INVALID;
  const double b1 = 1.0 - a0;
  double Ry = state[0], Rx = state[1];
  bool first = state[2] == 0.0;
  for (int i = 0; i < n; ++i) {
    const double ry = r[2 * i], rx = r[2 * i + 1];
    if (first) {  // Eq. 10 with R_{-1} = 0: R_0 = a0 r_0, never rate-limited
      Ry = a0 * ry;
      Rx = a0 * rx;
      first = false;
    } else if (rate_limit > 0.0) {  // Eq. 11-12
      double dy = a0 * ry + (b1 - 1.0) * Ry, dx = a0 * rx + (b1 - 1.0) * Rx;
      const double L = std::hypot(dy, dx);
      if (L > rate_limit) {
        dy *= rate_limit / L;
        dx *= rate_limit / L;
      }
      Ry += dy;
      Rx += dx;
    } else {  // Eq. 10
      Ry = a0 * ry + b1 * Ry;
      Rx = a0 * rx + b1 * Rx;
    }
    out[2 * i] = ry - Ry;
    out[2 * i + 1] = rx - Rx;
  }
  state[0] = Ry;
  state[1] = Rx;
  state[2] += (double)n;
  return CCPT_OK;
}

int ccpt_stage_times(ccpt_ctx* ctx, double* ms, int* launches, int n_stages, int reset) {
  if (!ctx || n_stages < 0 || (n_stages > 0 && (!ms || !launches))) return CCPT_E_INVALID;
  for (int i = 0; i < n_stages; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (auto& sp : ctx->spans) {
    HIP_CHECK(ctx, hipEventSynchronize(sp.b));
    float t = 0.f;
    HIP_CHECK(ctx, hipEventElapsedTime(&t, sp.a, sp.b));
    if (sp.stage >= 0 && sp.stage < n_stages) {
      ms[sp.stage] += t;
      launches[sp.stage] += 1;
    }
  }
  if (reset) {
    for (auto& sp : ctx->spans) {
      ctx->ev_pool.push_back(sp.a);
      ctx->ev_pool.push_back(sp.b);
    }
    ctx->spans.clear();
  }
  return CCPT_OK;
}

// Event-timed average of `reps` calls of ccpt_track_batch (one untimed call
// first: allocations and graph captures); a negative value if a call failed.
static float time_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, ccpt_result* out,
                        void* stream, hipEvent_t e0, hipEvent_t e1, int reps) {
  hipStream_t s = (hipStream_t)stream;
  if (ccpt_track_batch(ctx, rois, n, out, stream) != CCPT_OK) return -1.f;
  if (hipEventRecord(e0, s) != hipSuccess) return -1.f;
  for (int r = 0; r < reps; ++r)
    if (ccpt_track_batch(ctx, rois, n, out, stream) != CCPT_OK) return -1.f;
  float ms = 0.f;
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    return -1.f;
  return ms / reps;
}

// Coordinate search over the launch plan of one shape code: chunk sizes, then
// the block plans that apply to the shape (FP32 split-K threshold; for
// 256x256 the one-kernel correlation threshold), then chunk sizes again if
// a block plan changed; every candidate timed on the whole call.
static void tune_shape(ccpt_ctx* ctx, int code, int count, const ccpt_roi* rois, int n,
                       ccpt_result* out, void* stream, hipEvent_t e0, hipEvent_t e1,
                       float& best_ms) {
  Schedule& sc = ctx->sched[code];
  auto trial = [&](Schedule cand) {
    const Schedule keep = sc;
    sc = cand;
    drop_graphs(ctx);
    const float ms = time_batch(ctx, rois, n, out, stream, e0, e1, 3);
    if (ms >= 0.f && ms < best_ms) {
      best_ms = ms;
      return true;
    }
    sc = keep;
    return false;
  };
  const int cands[] = {16, 32, 64, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 4096};
  auto sweep_chunks = [&]() {
    for (int c : cands) {
      if (c > count && c != cands[0]) break;
      if (frame_ws_bytes(code, ctx->o.precision) * (size_t)std::min(c, count) > ((size_t)8 << 30))
        break;
      Schedule cand = sc;
      cand.chunk = c;
      (void)trial(cand);
    }
  };
  sweep_chunks();
  bool changed = false;
  if (ctx->o.precision == CCPT_PREC_FP32)
    for (int sb : {0, kSplitMaxBlocks, 512}) {
      Schedule cand = sc;
      cand.split_blocks = sb;
      changed |= trial(cand);
    }
  if (code_ny(code) == 256 && code_nx(code) == 256 && !fp64(ctx))
    for (int fm : {1, kFusedMinFrames, 1 << 30}) {
      Schedule cand = sc;
      cand.fused_min = fm;
      changed |= trial(cand);
    }
  if (changed) sweep_chunks();
}

int ccpt_autotune(ccpt_ctx* ctx, int n, int batch, void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (batch < 1 || !supported_size(n)) return fail(ctx, CCPT_E_INVALID, "bad tuning shape");
  int rid = -1;
  for (int r = 0; r < (int)ctx->refs.size(); ++r)
    if (ctx->refs[r].n == n) {
      rid = r;
      break;
    }
  if (rid < 0) return fail(ctx, CCPT_E_NOREF, "no reference of size %d to tune with", n);
  int rc = set_device(ctx);
  if (rc) return rc;
  // every tuning frame is the reference image itself (timing does not depend on content)
  std::vector<ccpt_roi> rois(batch);
  for (auto& r : rois) r = ccpt_roi{ctx->refs[rid].img, n, n, n, CCPT_F32, rid};
  ccpt_result* out = nullptr;
  HIP_CHECK(ctx, hipMalloc(&out, (size_t)batch * sizeof(ccpt_result)));
  hipEvent_t e0, e1;
  HIP_CHECK(ctx, hipEventCreate(&e0));
  HIP_CHECK(ctx, hipEventCreate(&e1));
  const int saved_flags = ctx->o.flags;
  ctx->o.flags = 0;  // no graphs or profiling while tuning
  ctx->sched[n] = Schedule{};
  float best = 1e30f;
  tune_shape(ctx, n, batch, rois.data(), batch, out, stream, e0, e1, best);
  ctx->o.flags = saved_flags;
  drop_graphs(ctx);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  ctx->last_desc.clear();
  return CCPT_OK;
}

int ccpt_autotune_batch(ccpt_ctx* ctx, const ccpt_roi* rois, int n, void* stream) {
  if (!ctx) return CCPT_E_INVALID;
  if (n < 1 || !rois) return fail(ctx, CCPT_E_INVALID, "bad roi array");
  int rc = set_device(ctx);
  if (rc) return rc;
  Plan plan;
  rc = plan_rois(ctx, rois, n, plan);  // validates every roi
  if (rc) return rc;
  ccpt_result* out = nullptr;
  HIP_CHECK(ctx, hipMalloc(&out, (size_t)n * sizeof(ccpt_result)));
  hipEvent_t e0, e1;
  HIP_CHECK(ctx, hipEventCreate(&e0));
  HIP_CHECK(ctx, hipEventCreate(&e1));
  const int saved_flags = ctx->o.flags;
  ctx->o.flags = 0;  // no graphs or profiling while tuning
  const int ngroups = (int)plan.sig.size() / 2;
  auto tune_lanes = [&](float& best) {
    int best_l = ctx->lanes;
    for (int l = 1; l <= std::min(ngroups, kMaxLanes); ++l) {
      ctx->lanes = l;
      drop_graphs(ctx);
      const float ms = time_batch(ctx, rois, n, out, stream, e0, e1, 3);
      if (ms >= 0.f && ms < best) {
        best = ms;
        best_l = l;
      }
    }
    ctx->lanes = best_l;
  };
  float best = 1e30f;
  for (int gi = 0; gi < ngroups; ++gi) ctx->sched[plan.sig[2 * gi]] = Schedule{};
  ctx->lanes = 0;
  tune_lanes(best);
  // the shapes in the call's order (largest frames first), each plan timed on
  // the whole call with the others' plans fixed
  for (int gi = 0; gi < ngroups; ++gi)
    tune_shape(ctx, plan.sig[2 * gi], plan.sig[2 * gi + 1], rois, n, out, stream, e0, e1, best);
  tune_lanes(best);
  ctx->o.flags = saved_flags;
  drop_graphs(ctx);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  ctx->last_desc.clear();
  return CCPT_OK;
}

int ccpt_schedule(ccpt_ctx* ctx, int n, int* chunk, int set) {
  if (!ctx || !chunk) return CCPT_E_INVALID;
  if (!supported_size(n)) return fail(ctx, CCPT_E_UNSUPPORTED, "size %d", n);
  if (set) {
    if (*chunk < 0 || *chunk > (1 << 20)) return fail(ctx, CCPT_E_INVALID, "chunk %d", *chunk);
    ctx->sched[n].chunk = *chunk;
    drop_graphs(ctx);
  } else {
    *chunk = chunk_for(ctx, n);
  }
  return CCPT_OK;
}

int ccpt_get_plan(ccpt_ctx* ctx, int ny, int nx, ccpt_plan* p) {
  if (!ctx || !p) return CCPT_E_INVALID;
  const int code = shape_code(ny, nx);
  if (!code) return fail(ctx, CCPT_E_UNSUPPORTED, "shape %dx%d", ny, nx);
  p->chunk = chunk_for(ctx, code);
  p->split_blocks = split_blocks_for(ctx, code);
  p->fused_min = fused_min_for(ctx, code);
  return CCPT_OK;
}

int ccpt_set_plan(ccpt_ctx* ctx, int ny, int nx, const ccpt_plan* p) {
  if (!ctx || !p) return CCPT_E_INVALID;
  const int code = shape_code(ny, nx);
  if (!code) return fail(ctx, CCPT_E_UNSUPPORTED, "shape %dx%d", ny, nx);
  if (p->chunk < 0 || p->chunk > (1 << 20) || p->split_blocks < -1 || p->split_blocks > 512 ||
      p->fused_min < -1)
    return fail(ctx, CCPT_E_INVALID, "plan {%d, %d, %d}", p->chunk, p->split_blocks, p->fused_min);
  Schedule& sc = ctx->sched[code];
  sc.chunk = p->chunk;
  sc.split_blocks = p->split_blocks;
  sc.fused_min = p->fused_min;
  drop_graphs(ctx);
  return CCPT_OK;
}

int ccpt_lanes(ccpt_ctx* ctx, int* lanes, int set) {
  if (!ctx || !lanes) return CCPT_E_INVALID;
  if (set) {
    if (*lanes < 0 || *lanes > kMaxLanes) return fail(ctx, CCPT_E_INVALID, "lanes %d", *lanes);
    ctx->lanes = *lanes;
    drop_graphs(ctx);
  } else {
    *lanes = ctx->lanes > 0 ? ctx->lanes : kMaxLanes;
  }
  return CCPT_OK;
}

}  // extern "C"
