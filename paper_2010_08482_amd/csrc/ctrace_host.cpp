// Host side of the C ABI declared in include/ctrace.h: context, arena
// sub-allocation, impurity upload in the kernels' layout, validation,
// batching into arena-sized chunks and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctrace_internal.h"

using ctr::BatchArgs;
using ctr::DevImp;
using ctr::PanelRes;
using ctr::StrRec;

struct ctr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  size_t resident = 0;  // bytes of the arena held by the loaded impurity
  bool loaded = false;
  DevImp imp{};
  int n_sec = 0, nf = 0, nops = 0, max_dim = 0;
  double beta = 0.0;
  long long max_panels_per_cfg = 0;
  int grid = 0;
  int grid_split = 0;   // FP32-split, 6 slices
  int grid_split7 = 0;  // FP32-split, 7 slices
  int slices = 6;       // slices of the current FP32-split call
  int grid_wave = 0;  // wavefront-per-panel kernel (panels of 8 columns), 0 = not applicable
  int grid_wave_lazy = 0;  // its lazy form
  int grid_big = 0;   // streaming kernel
  int grid_group = 0;  // block-grouped rounds, 0 = not applicable
  int cw_group = 0;    // columns per grouped work item
  int rc_group = 0;    // rows per grouped product item (0: all rows of the block)
  int grid_rows = 0;   // the row-chunked grouped rounds (CTR_KERNEL_GROUPED_ROWS), any sector size
  int cw_rows = 0, rc_rows = 0;
  int grid_rsplit[2] = {0, 0};  // their FP32-split form, 6 and 7 slices
  int cw_rsplit = 0, rc_rsplit = 0;
  int last_kernel = 0, last_slices = 0;  // chain kernel and precision of the last trace call
  std::vector<int> h_dim, h_next;        // host copies of the sector table (footprint estimates)
  bool rows = false;   // the current grouped call runs the row-chunked items
  bool graph = false;  // the current grouped call launches its rounds as one HIP graph
  int gsplit = 0;      // slices of the current grouped call's FP32-split products (0: FP64)
  int galt = 0;        // grouped tile shape: 0 default, 1 the alternative (picked by ctr_tune)
  int tuned = 0;       // CTR_KERNEL_* picked by ctr_tune for FP64 batches (0 = none)
  int tuned_min_batch = 0;
  double grid_share = 1.0;  // fraction of each persistent grid launched (a serving lane's share)
  double* xbuf = nullptr;  // the streaming kernel's per-workgroup X buffers
  unsigned int* counter = nullptr;
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::string err;
};

namespace {

// Per-call scratch of ctr_trace_batch_device_static: a fixed device array
// instead of the context's arena.  Each device the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address hipGetSymbolAddress
// returned for the current device (g_scratch), taken once per device in
// ctr_create.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

ctr_status fail(ctr_ctx* ctx, ctr_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

// Workgroups of a persistent launch under the context's grid share: at least
// `floor` (the kernel's own minimum, at most g), at most the full grid g.
int shared_grid(const ctr_ctx* ctx, int g, int floor) {
  if (g <= 0 || ctx->grid_share >= 1.0) return g;
  const int n = (int)std::ceil(g * ctx->grid_share);
  return std::min(g, std::max(std::min(g, floor), n));
}

ctr_status hip_fail(ctr_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, CTR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

// Bump allocator over [base, end) of the arena.
struct Bump {
  char* base;
  size_t off, cap;
  void* take(size_t bytes) {
    size_t o = align_up(off);
    if (o + bytes > cap) return nullptr;
    off = o + bytes;
    return base + o;
  }
};

// Host-side check of one configuration (host-pointer entry points).
ctr_status check_config(ctr_ctx* ctx, long long n, const double* tau, const int32_t* op, long long cfg) {
  if (n < 0 || n > ctr::kMaxOps)
    return fail(ctx, CTR_ERR_ARG, "configuration " + std::to_string(cfg) + ": operator count outside [0, " +
                                      std::to_string(ctr::kMaxOps) + "]");
  for (long long i = 0; i < n; ++i) {
    if (!(tau[i] >= 0.0 && tau[i] < ctx->beta))
      return fail(ctx, CTR_ERR_RANGE, "configuration " + std::to_string(cfg) + ": tau outside [0, beta)");
    if (op[i] < 0 || op[i] >= ctx->nops)
      return fail(ctx, CTR_ERR_RANGE, "configuration " + std::to_string(cfg) + ": operator code out of range");
    if (i > 0 && !(tau[i] >= tau[i - 1]))
      return fail(ctx, CTR_ERR_UNSORTED, "configuration " + std::to_string(cfg) + ": tau not sorted");
  }
  return CTR_OK;
}

size_t scratch_per_cfg(const ctr_ctx* ctx) {
  // panels counted with the narrowest panel width any kernel uses (upper bound)
  return (size_t)ctx->n_sec * sizeof(StrRec) + 4 * sizeof(int) + 5 * sizeof(double) + sizeof(long long) +
         (size_t)ctx->max_panels_per_cfg * sizeof(PanelRes);
}

// Scratch for n_cfg configurations after `b`'s current offset.  Returns false if it does not fit.
bool carve(ctr_ctx* ctx, Bump& b, int n_cfg, BatchArgs& a) {
  a.n_cfg = n_cfg;
  a.rec = (StrRec*)b.take((size_t)n_cfg * ctx->n_sec * sizeof(StrRec));
  a.cfg_cnt = (int*)b.take((size_t)n_cfg * sizeof(int));
  a.cfg_flags = (int*)b.take((size_t)n_cfg * sizeof(int));
  a.cfg_nstr = (int*)b.take((size_t)n_cfg * sizeof(int));
  a.cfg_logB = (double*)b.take((size_t)n_cfg * sizeof(double));
  a.cfg_off = (long long*)b.take((size_t)(n_cfg + 1) * sizeof(long long));
  a.res = (PanelRes*)b.take((size_t)n_cfg * ctx->max_panels_per_cfg * sizeof(PanelRes));
  a.cfg_lthr = (double*)b.take((size_t)n_cfg * sizeof(double));
  a.cfg_bsum = (unsigned long long*)b.take((size_t)n_cfg * sizeof(unsigned long long));
  a.cfg_rej = (int*)b.take((size_t)n_cfg * sizeof(int));
  a.counter = ctx->counter;
  return a.rec && a.cfg_cnt && a.cfg_flags && a.cfg_nstr && a.cfg_logB && a.cfg_off && a.res && a.cfg_lthr &&
         a.cfg_bsum && a.cfg_rej;
}

enum class Kernel { Wave, Block, Stream, Group };

// Smallest batch for which AUTO takes the block-grouped rounds: below it the
// per-round launches cost more than the shared block reads save (f-shell,
// 327-state sectors, host arrays: even at 32 configurations, grouped 21%
// faster at 64 and 35% at 128).
constexpr int kGroupMinBatch = 48;

// Block-grouped rounds for the configurations of `a` (scratch after `b`'s
// offset).  Returns CTR_ERR_OOM, with nothing enqueued past the plan, if the
// carried matrices of the surviving strings do not fit the arena.
ctr_status enqueue_grouped(ctr_ctx* ctx, BatchArgs& a, Bump& b, const ctr::HistArgs* hist) {
  a.panel = ctr::kGroupPanel;
  hipError_t e = ctr::launch_plan(ctx->imp, a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "plan kernel");
  if ((e = ctr::launch_scan(a, ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "scan kernel");
  ctr::GroupArgs g{};
  const long long max_s = (long long)a.n_cfg * ctx->n_sec;
  g.s_cfg = (int*)b.take((size_t)max_s * sizeof(int));
  g.s_rec = (int*)b.take((size_t)max_s * sizeof(int));
  g.s_width = (int*)b.take((size_t)max_s * sizeof(int));
  g.s_n = (int*)b.take((size_t)max_s * sizeof(int));
  g.s_colbase = (long long*)b.take((size_t)max_s * sizeof(long long));
  g.info = (long long*)b.take(8 * sizeof(long long));
  if (!g.s_cfg || !g.s_rec || !g.s_width || !g.s_n || !g.s_colbase || !g.info)
    return fail(ctx, CTR_ERR_OOM, "arena too small");
  g.cw_step = ctx->gsplit ? ctx->cw_rsplit : ctx->rows ? ctx->cw_rows : ctx->cw_group;
  g.cw_close = ctr::kGroupCloseCols;
  g.rchunk = ctx->gsplit ? ctx->rc_rsplit : ctx->rows ? ctx->rc_rows : ctx->rc_group;
  if ((e = ctr::launch_group_prepare(ctx->imp, a, g, max_s, ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "grouped prepare kernels");
  long long info[5] = {0, 0, 0, 0, 0};
  HIP_TRY(ctx, hipMemcpyAsync(info, g.info, sizeof(info), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  g.S = info[0];
  g.T = info[1];
  g.R = (int)info[2];
  g.CS = info[3];
  g.NI = info[4];
  if (g.T >= (1LL << 31) || g.S >= (1LL << 31)) return fail(ctx, CTR_ERR_OOM, "batch too large for one chunk");
  const long long NK = 2LL * ctx->n_sec * ctx->nops;
  const long long R = std::max(g.R, 1);
  const int planes = ctx->imp.is_complex ? 2 : 1;
  const size_t xdoubles = (size_t)std::max(g.T, 1LL) * ctx->imp.xrows * planes;
  g.hist = (int*)b.take((size_t)(R * NK) * sizeof(int));
  g.hcols = (int*)b.take((size_t)(R * NK) * sizeof(int));
  g.cursor = (int*)b.take((size_t)(R * NK) * sizeof(int));
  g.gstart = (int*)b.take((size_t)(R * (NK + 1)) * sizeof(int));
  g.istart = (int*)b.take((size_t)(R * (NK + 1)) * sizeof(int));
  g.n_items = (int*)b.take((size_t)R * sizeof(int));
  g.counters = (unsigned int*)b.take((size_t)R * ctr::kGroupCounters * 32 * sizeof(unsigned int));
  g.sorted = (int*)b.take((size_t)(R * std::max(g.S, 1LL)) * sizeof(int));
  g.colpref = (int*)b.take((size_t)(R * std::max(g.S, 1LL)) * sizeof(int));
  g.X[0] = (double*)b.take(xdoubles * sizeof(double));
  g.X[1] = (double*)b.take(xdoubles * sizeof(double));
  g.colexp = (int*)b.take((size_t)std::max(g.T, 1LL) * sizeof(int));
  g.colres = (PanelRes*)b.take((size_t)std::max(g.T, 1LL) * sizeof(PanelRes));
  g.rcols = (long long*)b.take((size_t)R * sizeof(long long));
  g.rcoloff = (long long*)b.take((size_t)R * sizeof(long long));
  g.ritemoff = (long long*)b.take((size_t)R * sizeof(long long));
  g.item_key = (int*)b.take((size_t)std::max(g.NI, 1LL) * sizeof(int));
  g.colg = (int*)b.take((size_t)std::max(g.CS, 1LL) * sizeof(int));
  g.colaux = (double*)b.take((size_t)std::max(g.CS, 1LL) * sizeof(double));
  g.epend = g.rchunk > 0 ? (int*)b.take((size_t)3 * std::max(g.T, 1LL) * sizeof(int)) : nullptr;
  if (!g.hist || !g.hcols || !g.cursor || !g.gstart || !g.istart || !g.n_items || !g.counters || !g.sorted ||
      !g.colpref || !g.X[0] || !g.X[1] || !g.colexp || !g.colres || !g.rcols || !g.rcoloff || !g.ritemoff ||
      !g.item_key || !g.colg || !g.colaux || (g.rchunk > 0 && !g.epend))
    return fail(ctx, CTR_ERR_OOM, "arena too small for the grouped rounds");
  HIP_TRY(ctx, hipMemsetAsync(g.rcols, 0, (size_t)R * sizeof(long long), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.n_items, 0, (size_t)R * sizeof(int), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.hist, 0, (size_t)(R * NK) * sizeof(int), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.hcols, 0, (size_t)(R * NK) * sizeof(int), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.cursor, 0, (size_t)(R * NK) * sizeof(int), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.counters, 0, (size_t)R * ctr::kGroupCounters * 32 * sizeof(unsigned int), ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(g.colres, 0, (size_t)std::max(g.T, 1LL) * sizeof(PanelRes), ctx->stream));
  if ((e = ctr::launch_group_schedule(ctx->imp, a, g, ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "grouped schedule kernels");
  ctx->last_kernel = g.rchunk > 0 ? CTR_KERNEL_GROUPED_ROWS : CTR_KERNEL_GROUPED;
  ctx->last_slices = ctx->gsplit;
  if (ctx->graph && g.R > 1) {
    // one kernel node per round, each depending on the one before
    const int grid = ctx->gsplit ? ctx->grid_rsplit[ctx->gsplit == 7] : ctx->rows ? ctx->grid_rows : ctx->grid_group;
    hipGraph_t graph = nullptr;
    HIP_TRY(ctx, hipGraphCreate(&graph, 0));
    struct GraphGuard {
      hipGraph_t g;
      hipGraphExec_t x = nullptr;
      ~GraphGuard() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
      }
    } guard{graph};
    hipGraphNode_t prev = nullptr;
    std::vector<int> rounds(g.R);
    for (int r = 1; r < g.R; ++r) {
      rounds[r] = r;
      hipKernelNodeParams kp{};
      void* args[] = {&ctx->imp, &a, &g, &rounds[r]};
      if ((e = ctr::group_round_node(ctx->imp, g, shared_grid(ctx, grid, ctr::kGroupCounters),
                                     ctx->rows || ctx->gsplit ? 2 : ctx->galt, ctx->gsplit, args, &kp)) != hipSuccess)
        return hip_fail(ctx, e, "grouped round node");
      hipGraphNode_t node = nullptr;
      HIP_TRY(ctx, hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
      prev = node;
    }
    HIP_TRY(ctx, hipGraphInstantiate(&guard.x, graph, nullptr, nullptr, 0));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->timing) {
      HIP_TRY(ctx, hipEventCreate(&t0));
      HIP_TRY(ctx, hipEventCreate(&t1));
      HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
    }
    HIP_TRY(ctx, hipGraphLaunch(guard.x, ctx->stream));
    if (ctx->timing) {
      HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
      ctx->events.emplace_back(t0, t1);
    }
    // the executable graph is released once its launch has run
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  for (int r = 1; r < g.R && !ctx->graph; ++r) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->timing) {
      HIP_TRY(ctx, hipEventCreate(&t0));
      HIP_TRY(ctx, hipEventCreate(&t1));
      HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
    }
    const int grid = ctx->gsplit ? ctx->grid_rsplit[ctx->gsplit == 7] : ctx->rows ? ctx->grid_rows : ctx->grid_group;
    if ((e = ctr::launch_group_round(ctx->imp, a, g, r, shared_grid(ctx, grid, ctr::kGroupCounters),
                                     ctx->rows || ctx->gsplit ? 2 : ctx->galt, ctx->gsplit, ctx->stream)) != hipSuccess)
      return hip_fail(ctx, e, "grouped round kernel");
    if (ctx->timing) {
      HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
      ctx->events.emplace_back(t0, t1);
    }
  }
  if ((e = ctr::launch_group_combine(ctx->imp, a, g, ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "grouped combine kernel");
  if (hist) {
    ctr::HistArgs h = *hist;
    h.vals = g.colres;
    h.colbase = g.s_colbase;
    if ((e = ctr::launch_hist(ctx->imp, a, h, ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "histogram kernel");
  }
  return CTR_OK;
}

ctr_status enqueue(ctr_ctx* ctx, BatchArgs& a, bool plan_only, bool split, Kernel kind, Bump* b,
                   const ctr::HistArgs* hist = nullptr) {
  if (kind == Kernel::Group && !plan_only) return enqueue_grouped(ctx, a, *b, hist);
  a.panel = kind == Kernel::Wave ? ctr::kWavePanelHost : ctr::kPanel;
  hipError_t e = ctr::launch_plan(ctx->imp, a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "plan kernel");
  if (plan_only) return CTR_OK;
  e = ctr::launch_scan(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "scan kernel");
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (ctx->timing) {
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
  }
  ctx->last_kernel = kind == Kernel::Wave ? CTR_KERNEL_WAVE : kind == Kernel::Block ? CTR_KERNEL_BLOCK : CTR_KERNEL_STREAM;
  ctx->last_slices = split ? ctx->slices : 0;
  switch (kind) {
    case Kernel::Wave:
      e = ctr::launch_chain_wave(ctx->imp, a, shared_grid(ctx, a.log_thr ? ctx->grid_wave_lazy : ctx->grid_wave, 1),
                                 ctx->stream);
      break;
    case Kernel::Block:
      e = ctr::launch_chain(ctx->imp, a, split ? ctx->slices : 0,
                            shared_grid(ctx, split ? (ctx->slices == 7 ? ctx->grid_split7 : ctx->grid_split) : ctx->grid, 1),
                            ctx->stream);
      break;
    case Kernel::Stream:
      e = ctr::launch_chain_big(ctx->imp, a, ctx->xbuf, shared_grid(ctx, ctx->grid_big, 1), ctx->stream);
      break;
    case Kernel::Group: e = hipErrorInvalidValue; break;  // handled by enqueue_grouped
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "chain kernel");
  if (ctx->timing) {
    HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
    ctx->events.emplace_back(t0, t1);
  }
  e = ctr::launch_combine(ctx->imp, a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "combine kernel");
  if (hist) {
    ctr::HistArgs h = *hist;
    h.vals = a.res;
    h.colbase = nullptr;
    if ((e = ctr::launch_hist(ctx->imp, a, h, ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "histogram kernel");
  }
  return CTR_OK;
}

ctr_status ready(ctr_ctx* ctx) {
  if (!ctx) return CTR_ERR_ARG;
  if (!ctx->loaded) return fail(ctx, CTR_ERR_STATE, "no impurity loaded");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  ctx->err.clear();
  return CTR_OK;
}

ctr_status check_opts(ctr_ctx* ctx, const ctr_opts* opts, bool* split, Kernel* kind, long long n_cfg = 1,
                      bool lazy = false) {
  *split = false;
  int want = CTR_KERNEL_AUTO;
  if (opts) {
    if (opts->flags & ~CTR_OPT_GRAPH) return fail(ctx, CTR_ERR_ARG, "unknown ctr_opts.flags bits");
    if (opts->precision == CTR_FP32_SPLIT) {
      if (opts->slices != 0 && opts->slices != 6 && opts->slices != 7)
        return fail(ctx, CTR_ERR_UNSUPPORTED, "CTR_FP32_SPLIT supports 6 or 7 slices of 8 bits (slices = 0, 6 or 7)");
      *split = true;
      ctx->slices = opts->slices == 7 ? 7 : 6;
    } else if (opts->precision != CTR_FP64) {
      return fail(ctx, CTR_ERR_ARG, "unknown precision");
    }
    want = opts->kernel;
    if (want < CTR_KERNEL_AUTO || want > CTR_KERNEL_GROUPED_ROWS) return fail(ctx, CTR_ERR_ARG, "unknown kernel");
  }
  ctx->rows = false;
  ctx->gsplit = 0;
  ctx->graph = opts && (opts->flags & CTR_OPT_GRAPH);
  // grouped rounds with a threshold: the plan's bound rejects, strings are not refined while they run
  const bool group_ok = !*split && ctx->grid_group > 0;
  // FP32-split products in grouped rounds: the row-chunked items
  const bool rsplit_ok = *split && ctx->grid_rsplit[ctx->slices == 7] > 0;
  const bool wave_ok = !*split && ctx->grid_wave > 0;
  const bool block_ok = (*split ? (ctx->slices == 7 ? ctx->grid_split7 : ctx->grid_split) : ctx->grid) > 0;
  const bool stream_ok = !*split && ctx->grid_big > 0;
  switch (want) {
    case CTR_KERNEL_AUTO:
      if (ctx->tuned && !*split && !lazy && n_cfg >= ctx->tuned_min_batch) {
        *kind = ctx->tuned == CTR_KERNEL_WAVE     ? Kernel::Wave
                : ctx->tuned == CTR_KERNEL_BLOCK  ? Kernel::Block
                : ctx->tuned == CTR_KERNEL_STREAM ? Kernel::Stream
                                                  : Kernel::Group;
        return CTR_OK;
      }
      // sectors <= 128 states: the per-string wavefront kernel is as fast as
      // the grouped rounds; above, the grouped rounds win on batches
      if (rsplit_ok && (n_cfg >= kGroupMinBatch || !block_ok)) {
        ctx->gsplit = ctx->slices;
        *kind = Kernel::Group;
      } else if (wave_ok) *kind = Kernel::Wave;
      // row-chunked rounds (sectors above 384 states) beat the streaming kernel from one configuration on
      // (crystal-field f-shell: 170 against 1049 ms for one, 3.4 against 4.7 s for 48)
      else if (group_ok && (n_cfg >= kGroupMinBatch || ctx->rc_group > 0)) *kind = Kernel::Group;
      else if (block_ok) *kind = Kernel::Block;
      else if (stream_ok) *kind = Kernel::Stream;
      else return fail(ctx, CTR_ERR_UNSUPPORTED, "no chain kernel can run this impurity in this precision");
      return CTR_OK;
    case CTR_KERNEL_WAVE:
      if (!wave_ok) return fail(ctx, CTR_ERR_UNSUPPORTED, "wavefront kernel needs FP64 and sectors <= 128 states");
      *kind = Kernel::Wave;
      return CTR_OK;
    case CTR_KERNEL_BLOCK:
      if (!block_ok) return fail(ctx, CTR_ERR_UNSUPPORTED, "the panel of the largest sector does not fit LDS");
      *kind = Kernel::Block;
      return CTR_OK;
    case CTR_KERNEL_STREAM:
      if (!stream_ok) return fail(ctx, CTR_ERR_UNSUPPORTED, "streaming kernel runs FP64 only");
      *kind = Kernel::Stream;
      return CTR_OK;
    case CTR_KERNEL_GROUPED_ROWS:
    default:
      // FP32-split grouped calls run the row-chunked items
      if (*split) {
        if (!rsplit_ok) return fail(ctx, CTR_ERR_UNSUPPORTED, "no grouped FP32-split kernel for this impurity");
        ctx->gsplit = ctx->slices;
      } else if (want == CTR_KERNEL_GROUPED_ROWS) {
        if (ctx->grid_rows <= 0) return fail(ctx, CTR_ERR_UNSUPPORTED, "row-chunked rounds do not fit the device");
        ctx->rows = true;
      } else if (!group_ok) {
        return fail(ctx, CTR_ERR_UNSUPPORTED, "grouped rounds do not fit the device");
      }
      *kind = Kernel::Group;
      return CTR_OK;
  }
}

// The kernel AUTO takes when the grouped rounds do not fit the arena.
Kernel per_string_kernel(const ctr_ctx* ctx) {
  if (ctx->grid_wave > 0) return Kernel::Wave;
  if (ctx->grid > 0) return Kernel::Block;
  return Kernel::Stream;
}

// Host-pointer batch: validates, then runs arena-sized chunks; `mode` 0 =
// traces, 1 = bounds only (out_bound), thresholds optional.
// Label histogram requested with a host batch: host label table and output.
struct HistReq {
  const int32_t* label;  // [n_sec]
  int32_t n_labels;
  double* hist;          // [n_cfg][n_labels] complex
};

ctr_status host_batch(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau, const int32_t* op,
                      const double* log_thr, ctr_value* out, double* out_bound, int mode, bool split,
                      Kernel kind, BatchArgs* last = nullptr, bool auto_kind = false, const HistReq* hr = nullptr) {
  if (n_cfg < 0 || (n_cfg > 0 && (!offsets || (!out && !out_bound))))
    return fail(ctx, CTR_ERR_ARG, "null argument");
  if (n_cfg == 0) return CTR_OK;
  if (offsets[0] != 0) return fail(ctx, CTR_ERR_ARG, "offsets[0] must be 0");
  for (int32_t c = 0; c < n_cfg; ++c) {
    const long long n = offsets[c + 1] - offsets[c];
    if (n > 0 && (!tau || !op)) return fail(ctx, CTR_ERR_ARG, "null tau/op");
    ctr_status s = check_config(ctx, n, tau + offsets[c], op + offsets[c], c);
    if (s != CTR_OK) return s;
  }
  const size_t per_cfg = scratch_per_cfg(ctx) + sizeof(long long) + sizeof(ctr_value) + sizeof(double) + 64 +
                        (hr ? (size_t)hr->n_labels * 2 * sizeof(double) : 0);
  int32_t c0 = 0;
  int32_t cap = n_cfg;  // chunk cap, halved while the grouped rounds do not fit
  std::vector<long long> offs;
  while (c0 < n_cfg) {
    // largest chunk that fits the free arena
    const size_t free_bytes = ctx->arena_bytes - ctx->resident;
    int32_t c1 = c0;
    size_t need = 8 * kAlign;
    while (c1 < n_cfg && c1 - c0 < cap) {
      const size_t more = per_cfg + (size_t)(offsets[c1 + 1] - offsets[c1]) * (sizeof(double) + sizeof(int32_t));
      if (need + more > free_bytes) break;
      need += more;
      ++c1;
    }
    if (c1 == c0) return fail(ctx, CTR_ERR_OOM, "arena too small for one configuration");
    const int32_t m = c1 - c0;
    const long long ops0 = offsets[c0], nops = offsets[c1] - offsets[c0];
    Bump b{ctx->arena, ctx->resident, ctx->arena_bytes};
    BatchArgs a{};
    long long* d_offs = (long long*)b.take((size_t)(m + 1) * sizeof(long long));
    double* d_tau = (double*)b.take((size_t)std::max<long long>(nops, 1) * sizeof(double));
    int* d_op = (int*)b.take((size_t)std::max<long long>(nops, 1) * sizeof(int));
    ctr_value* d_out = (ctr_value*)b.take((size_t)m * sizeof(ctr_value));
    double* d_thr = log_thr ? (double*)b.take((size_t)m * sizeof(double)) : nullptr;
    ctr::HistArgs h{};
    if (hr) {
      h.label = (const int*)b.take((size_t)ctx->n_sec * sizeof(int));
      h.n_labels = hr->n_labels;
      h.hist = (double*)b.take((size_t)m * hr->n_labels * 2 * sizeof(double));
      if (!h.label || !h.hist) return fail(ctx, CTR_ERR_OOM, "arena too small");
      HIP_TRY(ctx, hipMemcpyAsync((void*)h.label, hr->label, (size_t)ctx->n_sec * sizeof(int), hipMemcpyHostToDevice,
                                  ctx->stream));
    }
    if (!d_offs || !d_tau || !d_op || !d_out || (log_thr && !d_thr) || !carve(ctx, b, m, a))
      return fail(ctx, CTR_ERR_OOM, "arena too small");
    offs.resize(m + 1);
    for (int32_t i = 0; i <= m; ++i) offs[i] = offsets[c0 + i] - ops0;
    HIP_TRY(ctx, hipMemcpyAsync(d_offs, offs.data(), (m + 1) * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
    if (nops > 0) {
      HIP_TRY(ctx, hipMemcpyAsync(d_tau, tau + ops0, nops * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      HIP_TRY(ctx, hipMemcpyAsync(d_op, op + ops0, nops * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    }
    if (d_thr) HIP_TRY(ctx, hipMemcpyAsync(d_thr, log_thr + c0, m * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    a.offsets = d_offs;
    a.tau = d_tau;
    a.op = d_op;
    a.log_thr = d_thr;
    a.out = d_out;
    ctr_status s = enqueue(ctx, a, mode == 1, split, kind, &b, hr ? &h : nullptr);
    if (s == CTR_ERR_OOM && kind == Kernel::Group) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      if (m > 1) {
        cap = m / 2;
      } else if (auto_kind) {
        kind = per_string_kernel(ctx);
        cap = n_cfg;
      } else {
        return s;
      }
      ctx->err.clear();
      continue;
    }
    if (s != CTR_OK) return s;
    if (mode == 1) {
      HIP_TRY(ctx, hipMemcpyAsync(out_bound + c0, a.cfg_logB, m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    } else {
      HIP_TRY(ctx, hipMemcpyAsync(out + c0, d_out, m * sizeof(ctr_value), hipMemcpyDeviceToHost, ctx->stream));
      if (hr)
        HIP_TRY(ctx, hipMemcpyAsync(hr->hist + (size_t)c0 * hr->n_labels * 2, h.hist,
                                    (size_t)m * hr->n_labels * 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (last) *last = a;
    c0 = c1;
  }
  return CTR_OK;
}

}  // namespace

namespace ctr {

bool context_loaded(const ctr_ctx* ctx) { return ctx && ctx->loaded; }
double context_beta(const ctr_ctx* ctx) { return ctx->beta; }
int context_nops(const ctr_ctx* ctx) { return ctx->nops; }
size_t context_free_scratch(const ctr_ctx* ctx) { return ctx->arena_bytes - ctx->resident; }
void context_set_grid_share(ctr_ctx* ctx, double share) { ctx->grid_share = share; }
double request_flops(const ctr_ctx* ctx, long long n_ops, const int32_t* op) {
  // block products of every surviving string rotated to its narrowest sector: 2 (8 complex) flops per
  // multiply-add, width x d_out x d_in per operator
  const double c = ctx->imp.is_complex ? 8.0 : 2.0;
  double total = 0.0;
  std::vector<int> path((size_t)std::max(n_ops, 0LL) + 1);
  for (int q0 = 0; q0 < ctx->n_sec; ++q0) {
    int q = q0, w = ctx->h_dim[q0];
    path[0] = q0;
    long long i = 0;
    for (; i < n_ops && q >= 0; ++i) {
      q = ctx->h_next[(size_t)q * ctx->nops + op[i]];
      path[i + 1] = q;
      if (q >= 0) w = std::min(w, ctx->h_dim[q]);
    }
    if (q != q0 || i < n_ops) continue;
    double steps = 0.0;
    for (long long j = 0; j < n_ops; ++j) steps += (double)ctx->h_dim[path[j]] * ctx->h_dim[path[j + 1]];
    total += c * w * steps;
  }
  return total;
}

size_t request_scratch_bytes(const ctr_ctx* ctx, long long n_ops, const int32_t* op) {
  size_t bytes = scratch_per_cfg(ctx) + sizeof(long long) + sizeof(ctr_value) + sizeof(double) + 64 +
                 (size_t)n_ops * (sizeof(double) + sizeof(int32_t));
  if (ctx->grid_group <= 0 || !op) return bytes;
  // grouped rounds: every surviving string's columns (its narrowest sector) stay resident as two
  // copies of the carried matrix, plus per-column and per-column-step schedule entries
  long long cols = 0;
  for (int q0 = 0; q0 < ctx->n_sec; ++q0) {
    int q = q0, w = ctx->h_dim[q0];
    for (long long i = 0; i < n_ops && q >= 0; ++i) {
      q = ctx->h_next[(size_t)q * ctx->nops + op[i]];
      if (q >= 0) w = std::min(w, ctx->h_dim[q]);
    }
    if (q == q0) cols += w;
  }
  const size_t planes = ctx->imp.is_complex ? 2 : 1;
  return bytes + (size_t)cols * (2 * (size_t)ctx->imp.xrows * planes * sizeof(double) + 64) +
         (size_t)cols * (size_t)std::max(n_ops, 1LL) * (sizeof(int) + sizeof(double));
}

}  // namespace ctr

extern "C" {

const char* ctr_version(void) { return "ctrace 0.1 (gfx950, FP64 MFMA)"; }

const char* ctr_status_string(ctr_status s) {
  switch (s) {
    case CTR_OK: return "CTR_OK";
    case CTR_ERR_ARG: return "CTR_ERR_ARG";
    case CTR_ERR_OOM: return "CTR_ERR_OOM";
    case CTR_ERR_DEVICE: return "CTR_ERR_DEVICE";
    case CTR_ERR_UNSORTED: return "CTR_ERR_UNSORTED";
    case CTR_ERR_RANGE: return "CTR_ERR_RANGE";
    case CTR_ERR_STATE: return "CTR_ERR_STATE";
    case CTR_ERR_UNSUPPORTED: return "CTR_ERR_UNSUPPORTED";
    case CTR_ERR_BUSY: return "CTR_ERR_BUSY";
  }
  return "unknown status";
}

const char* ctr_last_error(const ctr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ctr_status ctr_create(int device, void* arena, size_t arena_bytes, void* hip_stream, ctr_ctx** out) {
  if (!out || !arena) return CTR_ERR_ARG;
  *out = nullptr;
  if (arena_bytes < (1u << 20)) return CTR_ERR_ARG;
  if (((uintptr_t)arena) % kAlign) return CTR_ERR_ARG;
  if (device < 0 || device >= kMaxDevices) return CTR_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return CTR_ERR_DEVICE;
  {
    // device address of this device's static scratch array, once per device
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CTR_ERR_DEVICE;
      g_scratch[device] = p;
    }
  }
  ctr_ctx* ctx = new ctr_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->arena = (char*)arena;
  ctx->arena_bytes = arena_bytes;
  *out = ctx;
  return CTR_OK;
}

void ctr_destroy(ctr_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& ev : ctx->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  delete ctx;
}

size_t ctr_arena_resident_bytes(const ctr_ctx* ctx) { return ctx ? ctx->resident : 0; }

ctr_status ctr_set_impurity(ctr_ctx* ctx, const ctr_impurity* imp) {
  if (!ctx) return CTR_ERR_ARG;
  if (!imp) return fail(ctx, CTR_ERR_ARG, "null impurity");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  ctx->loaded = false;
  ctx->resident = 0;
  const int nf = imp->n_flavors, ns = imp->n_sectors, nops = 2 * nf;
  if (!(imp->beta > 0.0) || nf < 1 || nf > 32 || ns < 1 || imp->reserved != 0)
    return fail(ctx, CTR_ERR_ARG, "beta, n_flavors or n_sectors out of range");
  if (!imp->sector_dim || !imp->energies || !imp->next || !imp->blocks)
    return fail(ctx, CTR_ERR_ARG, "null table");
  const bool cplx = imp->is_complex != 0;
  std::vector<int> dim(imp->sector_dim, imp->sector_dim + ns);
  int maxd = 0;
  for (int q = 0; q < ns; ++q) {
    if (dim[q] < 1) return fail(ctx, CTR_ERR_ARG, "sector dimension < 1");
    maxd = std::max(maxd, dim[q]);
  }
  std::vector<int> next(imp->next, imp->next + (size_t)ns * nops);
  for (int q = 0; q < ns; ++q)
    for (int f = 0; f < nf; ++f) {
      const int a = next[q * nops + 2 * f], c = next[q * nops + 2 * f + 1];
      if (a < -1 || a >= ns || c < -1 || c >= ns) return fail(ctx, CTR_ERR_ARG, "next entry out of range");
      if ((a >= 0) != (imp->blocks[q * nf + f] != nullptr))
        return fail(ctx, CTR_ERR_ARG, "block presence does not match next[q][2f]");
      if (a >= 0 && next[a * nops + 2 * f + 1] != q)
        return fail(ctx, CTR_ERR_ARG, "next table: c_f then c+_f does not return to the sector");
      if (c >= 0 && next[c * nops + 2 * f] != q)
        return fail(ctx, CTR_ERR_ARG, "next table: c+_f then c_f does not return to the sector");
    }
  if (ns > 32767) return fail(ctx, CTR_ERR_UNSUPPORTED, "more than 32767 sectors");
  // energies: global minimum, per-sector minimum, shifted and padded copies
  std::vector<double> emin(ns), esh;
  std::vector<int> eoff(ns);
  double E0 = INFINITY;
  {
    long long p = 0;
    for (int q = 0; q < ns; ++q) {
      double m = INFINITY;
      for (int i = 0; i < dim[q]; ++i) {
        const double e = imp->energies[p + i];
        if (!std::isfinite(e)) return fail(ctx, CTR_ERR_ARG, "non-finite energy");
        m = std::min(m, e);
      }
      emin[q] = m;
      E0 = std::min(E0, m);
      eoff[q] = (int)esh.size();
      for (int i = 0; i < ctr::pad16(dim[q]); ++i) esh.push_back(i < dim[q] ? imp->energies[p + i] - m : 0.0);
      p += dim[q];
    }
  }
  std::vector<double> lognorm((size_t)ns * nops, 0.0);
  if (imp->block_norm)
    for (int q = 0; q < ns; ++q)
      for (int f = 0; f < nf; ++f) {
        const double v = imp->block_norm[q * nf + f];
        if (next[q * nops + 2 * f] >= 0) {
          if (!(v > 0.0)) return fail(ctx, CTR_ERR_ARG, "block_norm must be > 0");
          lognorm[q * nops + 2 * f] = std::log(v);
          // c+_f leaving p = next[q][2f] is the adjoint of this block: same norm
          lognorm[next[q * nops + 2 * f] * nops + 2 * f + 1] = std::log(v);
        }
      }

  // block layout
  std::vector<long long> boff((size_t)ns * nops, -1);
  long long pool_doubles = 0;
  for (int q = 0; q < ns; ++q)
    for (int o = 0; o < nops; ++o) {
      const int t = next[q * nops + o];
      if (t < 0) continue;
      boff[q * nops + o] = pool_doubles;
      const long long sz = (long long)ctr::pad16(dim[t]) * ctr::pad4(dim[q]) * (cplx ? 2 : 1);
      pool_doubles += (sz + 31) & ~31LL;
    }

  // row exponents of every block (FP32-split scaling): pad16(d_out) int16 per block
  std::vector<long long> roff((size_t)ns * nops, -1);
  long long rexp_n = 0;
  for (int q = 0; q < ns; ++q)
    for (int o = 0; o < nops; ++o) {
      const int t = next[q * nops + o];
      if (t < 0) continue;
      roff[q * nops + o] = rexp_n;
      rexp_n += ctr::pad16(dim[t]);
    }
  std::vector<short> rexp((size_t)std::max(rexp_n, 1LL), 0);
  // nonzero 16 x 4 tiles of the blocks the wavefront kernel can run (at most 8 row tiles, 32 k-steps)
  std::vector<unsigned int> tmask((size_t)ns * nops * 8, 0xffffffffu);

  Bump b{ctx->arena, 0, ctx->arena_bytes};
  ctx->counter = (unsigned int*)b.take(sizeof(unsigned int));
  int* d_dim = (int*)b.take(ns * sizeof(int));
  int* d_next = (int*)b.take((size_t)ns * nops * sizeof(int));
  long long* d_boff = (long long*)b.take((size_t)ns * nops * sizeof(long long));
  double* d_emin = (double*)b.take(ns * sizeof(double));
  int* d_eoff = (int*)b.take(ns * sizeof(int));
  double* d_esh = (double*)b.take(esh.size() * sizeof(double));
  double* d_lognorm = (double*)b.take((size_t)ns * nops * sizeof(double));
  long long* d_roff = (long long*)b.take((size_t)ns * nops * sizeof(long long));
  short* d_rexp = (short*)b.take(rexp.size() * sizeof(short));
  double* d_pool = (double*)b.take((size_t)std::max(pool_doubles, 1LL) * sizeof(double));
  unsigned int* d_tmask = (unsigned int*)b.take(tmask.size() * sizeof(unsigned int));
  if (!ctx->counter || !d_dim || !d_next || !d_boff || !d_emin || !d_eoff || !d_esh || !d_lognorm || !d_pool ||
      !d_roff || !d_rexp || !d_tmask)
    return fail(ctx, CTR_ERR_OOM, "arena too small for the impurity (" +
                                      std::to_string((pool_doubles * 8) >> 20) + " MiB of blocks)");
  HIP_TRY(ctx, hipMemcpyAsync(d_dim, dim.data(), ns * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_next, next.data(), next.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_boff, boff.data(), boff.size() * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_emin, emin.data(), ns * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_eoff, eoff.data(), ns * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_esh, esh.data(), esh.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_lognorm, lognorm.data(), lognorm.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));

  // blocks: column-major, zero padded; creators are conjugate transposes of
  // the annihilator block leaving the target sector
  std::vector<double> stage;
  for (int q = 0; q < ns; ++q)
    for (int o = 0; o < nops; ++o) {
      const int t = next[q * nops + o];
      if (t < 0) continue;
      const int f = o >> 1, dag = o & 1;
      const int d_out = dim[t], d_in = dim[q];
      const int ld = ctr::pad16(d_out), kp = ctr::pad4(d_in);
      const size_t plane = (size_t)ld * kp;
      stage.assign(plane * (cplx ? 2 : 1), 0.0);
      if (!dag) {
        // annihilator leaving q: host block row-major d_out x d_in
        const void* src = imp->blocks[q * nf + f];
        for (int m = 0; m < d_out; ++m)
          for (int k = 0; k < d_in; ++k) {
            const size_t h = (size_t)m * d_in + k, dst = (size_t)k * ld + m;
            if (cplx) {
              const double* z = (const double*)src + 2 * h;
              stage[dst] = z[0];
              stage[plane + dst] = z[1];
            } else {
              stage[dst] = ((const double*)src)[h];
            }
          }
      } else {
        // creator leaving q = adjoint of the annihilator leaving t (d_in x d_out row-major)
        const void* src = imp->blocks[t * nf + f];
        for (int k = 0; k < d_in; ++k)
          for (int m = 0; m < d_out; ++m) {
            const size_t h = (size_t)k * d_out + m, dst = (size_t)k * ld + m;
            if (cplx) {
              const double* z = (const double*)src + 2 * h;
              stage[dst] = z[0];
              stage[plane + dst] = -z[1];
            } else {
              stage[dst] = ((const double*)src)[h];
            }
          }
      }
      for (int m = 0; m < ld; ++m) {
        double mx = 0.0;
        for (int k = 0; k < kp; ++k) {
          mx = std::max(mx, std::fabs(stage[(size_t)k * ld + m]));
          if (cplx) mx = std::max(mx, std::fabs(stage[plane + (size_t)k * ld + m]));
        }
        int ex = 0;
        if (mx > 0.0) std::frexp(mx, &ex);  // mx < 2^ex
        rexp[roff[q * nops + o] + m] = (short)std::max(-30000, std::min(30000, ex));
      }
      if (ld <= 128 && kp <= 128) {
        unsigned int* w = tmask.data() + (size_t)(q * nops + o) * 8;
        for (int tt = 0; tt < 8; ++tt) w[tt] = 0u;
        for (int k = 0; k < kp; ++k)
          for (int m = 0; m < ld; ++m) {
            const size_t a = (size_t)k * ld + m;
            if (stage[a] != 0.0 || (cplx && stage[plane + a] != 0.0)) w[m >> 4] |= 1u << (k >> 2);
          }
      }
      HIP_TRY(ctx, hipMemcpyAsync(d_pool + boff[q * nops + o], stage.data(), stage.size() * sizeof(double),
                                  hipMemcpyHostToDevice, ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
  HIP_TRY(ctx, hipMemcpyAsync(d_roff, roff.data(), roff.size() * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_rexp, rexp.data(), rexp.size() * sizeof(short), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_tmask, tmask.data(), tmask.size() * sizeof(unsigned int), hipMemcpyHostToDevice,
                              ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));

  ctx->imp.n_sec = ns;
  ctx->imp.nops = nops;
  ctx->imp.is_complex = cplx ? 1 : 0;
  ctx->imp.xrows = ctr::pad16(maxd);
  ctx->imp.next_lds = (ns * nops <= 16384 && ns < 32768) ? 1 : 0;
  ctx->imp.beta = imp->beta;
  ctx->imp.E0 = E0;
  ctx->imp.dim = d_dim;
  ctx->imp.next = d_next;
  ctx->imp.boff = d_boff;
  ctx->imp.emin = d_emin;
  ctx->imp.eoff = d_eoff;
  ctx->imp.esh = d_esh;
  ctx->imp.lognorm = d_lognorm;
  ctx->imp.pool = d_pool;
  ctx->imp.roff = d_roff;
  ctx->imp.rexp = d_rexp;
  ctx->imp.tmask = d_tmask;
  ctx->h_dim = dim;
  ctx->h_next = next;
  ctx->n_sec = ns;
  ctx->nf = nf;
  ctx->nops = nops;
  ctx->max_dim = maxd;
  ctx->beta = imp->beta;
  long long mp = 0;
  for (int q = 0; q < ns; ++q) mp += (dim[q] + ctr::kWavePanelHost - 1) / ctr::kWavePanelHost;
  ctx->max_panels_per_cfg = mp;
  ctx->grid = ctr::chain_grid(ctx->imp, ctx->device, 0, nullptr);
  ctx->grid_split = ctr::chain_grid(ctx->imp, ctx->device, 6, nullptr);
  ctx->grid_split7 = ctr::chain_grid(ctx->imp, ctx->device, 7, nullptr);
  ctx->grid_wave = ctr::wave_grid(ctx->imp, ctx->device, nullptr);
  ctx->grid_wave_lazy = ctr::wave_grid(ctx->imp, ctx->device, nullptr, true);
  ctx->grid_big = ctr::big_grid(ctx->imp, ctx->device, nullptr);
  ctx->cw_group = 0;
  ctx->rc_group = 0;
  ctx->galt = 0;
  ctx->grid_group = ctr::group_grid(ctx->imp, ctx->device, 0, &ctx->cw_group, &ctx->rc_group);
  ctx->grid_rows = ctr::group_grid(ctx->imp, ctx->device, 2, &ctx->cw_rows, &ctx->rc_rows);
  ctx->grid_rsplit[0] = ctr::group_grid(ctx->imp, ctx->device, 2, &ctx->cw_rsplit, &ctx->rc_rsplit, 6);
  ctx->grid_rsplit[1] = ctr::group_grid(ctx->imp, ctx->device, 2, &ctx->cw_rsplit, &ctx->rc_rsplit, 7);
  ctx->tuned = 0;
  ctx->tuned_min_batch = 0;
  ctx->xbuf = nullptr;
  if (ctx->grid_big > 0) {
    ctx->xbuf = (double*)b.take(ctr::big_xbuf_doubles(ctx->imp, ctx->grid_big) * sizeof(double));
    if (!ctx->xbuf) return fail(ctx, CTR_ERR_OOM, "arena too small for the streaming kernel's buffers");
  }
  if (ctx->grid <= 0 && ctx->grid_wave <= 0 && ctx->grid_big <= 0)
    return fail(ctx, CTR_ERR_UNSUPPORTED, "no chain kernel fits this impurity on the device");
  ctx->resident = align_up(b.off);
  ctx->loaded = true;
  return CTR_OK;
}

ctr_status ctr_trace_batch(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau, const int32_t* op,
                           const ctr_opts* opts, ctr_value* out) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, opts, &split, &kind, n_cfg)) != CTR_OK) return s;
  const bool auto_kind = !opts || opts->kernel == CTR_KERNEL_AUTO;
  return host_batch(ctx, n_cfg, offsets, tau, op, nullptr, out, nullptr, 0, split, kind, nullptr, auto_kind);
}

ctr_status ctr_tune(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau, const int32_t* op,
                    int32_t* chosen, double* ms_per_kernel) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  if (n_cfg < 1 || !offsets) return fail(ctx, CTR_ERR_ARG, "empty sample");
  if (ms_per_kernel)
    for (int k = 0; k < 5; ++k) ms_per_kernel[k] = -1.0;
  ctx->tuned = 0;
  std::vector<ctr_value> out(n_cfg);
  // candidates: every kernel, the grouped rounds in each of their tile shapes
  const int cands[5][2] = {{CTR_KERNEL_WAVE, 0}, {CTR_KERNEL_BLOCK, 0}, {CTR_KERNEL_STREAM, 0},
                           {CTR_KERNEL_GROUPED, 0}, {CTR_KERNEL_GROUPED, 1}};
  int best = 0, g_alt = 0;
  double best_ms = 0.0, g_ms = -1.0;
  const int grid0 = ctx->grid_group, cw0 = ctx->cw_group, rc0 = ctx->rc_group;
  // an error return leaves the grouped rounds in their default tile shape
  struct Restore {
    ctr_ctx* c;
    int grid, cw, rc;
    bool keep = false;
    ~Restore() {
      if (!keep) {
        c->galt = 0;
        c->grid_group = grid;
        c->cw_group = cw;
        c->rc_group = rc;
      }
    }
  } restore{ctx, grid0, cw0, rc0};
  for (const auto& cand : cands) {
    const int want = cand[0], alt = cand[1];
    if (want == CTR_KERNEL_GROUPED) {
      int cw = 0, rc = 0;
      const int grid = ctr::group_grid(ctx->imp, ctx->device, alt, &cw, &rc);
      if (grid <= 0) continue;
      ctx->galt = alt;
      ctx->grid_group = grid;
      ctx->cw_group = cw;
      ctx->rc_group = rc;
    }
    ctr_opts o{};
    o.kernel = want;
    bool split = false;
    Kernel kind = Kernel::Block;
    if (check_opts(ctx, &o, &split, &kind, n_cfg) != CTR_OK) continue;  // not applicable here
    ctx->err.clear();
    if ((s = host_batch(ctx, n_cfg, offsets, tau, op, nullptr, out.data(), nullptr, 0, false, kind)) != CTR_OK) {
      if (s == CTR_ERR_OOM) continue;  // its scratch does not fit: not a candidate
      return s;
    }
    hipEvent_t t0, t1;
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
    s = host_batch(ctx, n_cfg, offsets, tau, op, nullptr, out.data(), nullptr, 0, false, kind);
    HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
    HIP_TRY(ctx, hipEventSynchronize(t1));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (s != CTR_OK) return s;
    if (ms_per_kernel && (ms_per_kernel[want] < 0.0 || ms < ms_per_kernel[want])) ms_per_kernel[want] = ms;
    if (want == CTR_KERNEL_GROUPED && (g_ms < 0.0 || ms < g_ms)) {
      g_alt = alt;
      g_ms = ms;
    }
    if (!best || ms < best_ms) {
      best = want;
      best_ms = ms;
    }
  }
  // the grouped rounds keep their fastest tile shape
  ctx->galt = g_alt;
  ctx->grid_group = ctx->galt ? ctr::group_grid(ctx->imp, ctx->device, 1, &ctx->cw_group, &ctx->rc_group) : grid0;
  if (!ctx->galt) {
    ctx->cw_group = cw0;
    ctx->rc_group = rc0;
  }
  restore.keep = true;
  ctx->err.clear();
  if (!best) return fail(ctx, CTR_ERR_UNSUPPORTED, "no chain kernel ran the sample");
  ctx->tuned = best;
  ctx->tuned_min_batch = std::max(1, n_cfg / 4);
  if (chosen) *chosen = best;
  return CTR_OK;
}

ctr_status ctr_trace(ctr_ctx* ctx, int32_t n_ops, const double* tau, const int32_t* op, const ctr_opts* opts,
                     ctr_value* out) {
  if (n_ops < 0) return fail(ctx, CTR_ERR_ARG, "n_ops < 0");
  const int64_t offs[2] = {0, n_ops};
  return ctr_trace_batch(ctx, 1, offs, tau, op, opts, out);
}

ctr_status ctr_trace_lazy_batch(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau,
                                const int32_t* op, const double* log_threshold, const ctr_opts* opts,
                                ctr_value* out) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, opts, &split, &kind, n_cfg, true)) != CTR_OK) return s;
  if (n_cfg > 0 && !log_threshold) return fail(ctx, CTR_ERR_ARG, "null log_threshold");
  return host_batch(ctx, n_cfg, offsets, tau, op, log_threshold, out, nullptr, 0, split, kind);
}

ctr_status ctr_trace_lazy(ctr_ctx* ctx, int32_t n_ops, const double* tau, const int32_t* op, double log_threshold,
                          const ctr_opts* opts, ctr_value* out) {
  if (n_ops < 0) return fail(ctx, CTR_ERR_ARG, "n_ops < 0");
  const int64_t offs[2] = {0, n_ops};
  return ctr_trace_lazy_batch(ctx, 1, offs, tau, op, &log_threshold, opts, out);
}

ctr_status ctr_trace_histogram(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau,
                               const int32_t* op, const int32_t* sector_label, int32_t n_labels,
                               const ctr_opts* opts, ctr_value* out, double* hist) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, opts, &split, &kind, n_cfg)) != CTR_OK) return s;
  if (!sector_label || n_labels < 1 || n_labels > CTR_MAX_LABELS) return fail(ctx, CTR_ERR_ARG, "bad label table");
  if (n_cfg > 0 && (!hist || !out)) return fail(ctx, CTR_ERR_ARG, "null output");
  for (int q = 0; q < ctx->n_sec; ++q)
    if (sector_label[q] < 0 || sector_label[q] >= n_labels) return fail(ctx, CTR_ERR_RANGE, "sector label out of range");
  const HistReq hr{sector_label, n_labels, hist};
  const bool auto_kind = !opts || opts->kernel == CTR_KERNEL_AUTO;
  return host_batch(ctx, n_cfg, offsets, tau, op, nullptr, out, nullptr, 0, split, kind, nullptr, auto_kind, &hr);
}

ctr_status ctr_density_matrix(ctr_ctx* ctx, int32_t n_cfg, const int64_t* offsets, const double* tau,
                              const int32_t* op, const double* weight, ctr_value* out, double* rho) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  if (n_cfg < 1 || !offsets || !out || !rho) return fail(ctx, CTR_ERR_ARG, "null argument or empty batch");
  if (ctx->max_dim > ctr::kRdmMaxRows)
    return fail(ctx, CTR_ERR_UNSUPPORTED, "the density-matrix estimator handles sectors of at most " +
                                              std::to_string(ctr::kRdmMaxRows) + " states");
  // the traces first: every contribution is normalised by its configuration's weight
  if ((s = ctr_trace_batch(ctx, n_cfg, offsets, tau, op, nullptr, out)) != CTR_OK) return s;
  std::vector<long long> roff(ctx->n_sec);
  long long entries = 0;
  for (int q = 0; q < ctx->n_sec; ++q) {
    roff[q] = entries;
    entries += (long long)ctx->h_dim[q] * ctx->h_dim[q];
  }
  int slots = 1;
  for (int32_t c = 0; c < n_cfg; ++c) slots = std::max<long long>(slots, offsets[c + 1] - offsets[c]);
  const long long nops = offsets[n_cfg];
  Bump b{ctx->arena, ctx->resident, ctx->arena_bytes};
  long long* d_offs = (long long*)b.take((size_t)(n_cfg + 1) * sizeof(long long));
  double* d_tau = (double*)b.take((size_t)std::max(nops, 1LL) * sizeof(double));
  int* d_op = (int*)b.take((size_t)std::max(nops, 1LL) * sizeof(int));
  double* d_w = (double*)b.take((size_t)n_cfg * 2 * sizeof(double));
  double* d_wlog = (double*)b.take((size_t)n_cfg * sizeof(double));
  double* d_weight = (double*)b.take((size_t)n_cfg * 2 * sizeof(double));
  double* d_rho = (double*)b.take((size_t)entries * 2 * sizeof(double));
  long long* d_roff = (long long*)b.take((size_t)ctx->n_sec * sizeof(long long));
  BatchArgs a{};
  if (!d_offs || !d_tau || !d_op || !d_w || !d_wlog || !d_weight || !d_rho || !d_roff || !carve(ctx, b, n_cfg, a))
    return fail(ctx, CTR_ERR_OOM, "arena too small for the density-matrix batch");
  const size_t per_wg = ctr::rdm_buffer_doubles(ctx->imp, slots);
  const size_t left = b.cap - align_up(b.off);
  const int grid = (int)std::min<size_t>((size_t)ctr::rdm_grid(ctx->device), left / (per_wg * sizeof(double) + kAlign));
  double* d_buf = grid > 0 ? (double*)b.take((size_t)grid * per_wg * sizeof(double)) : nullptr;
  if (!d_buf) return fail(ctx, CTR_ERR_OOM, "arena too small for the density-matrix buffers");
  std::vector<double> w(2 * (size_t)n_cfg), wlog(n_cfg), wt(2 * (size_t)n_cfg);
  for (int32_t c = 0; c < n_cfg; ++c) {
    const bool skip = out[c].flags & (CTR_FLAG_ZERO | CTR_FLAG_REJECTED | CTR_FLAG_INVALID);
    w[2 * c] = skip ? 0.0 : out[c].re;
    w[2 * c + 1] = skip ? 0.0 : out[c].im;
    wlog[c] = out[c].log_scale + ctx->beta * ctx->imp.E0;
    wt[2 * c] = weight ? weight[2 * c] : 1.0;
    wt[2 * c + 1] = weight ? weight[2 * c + 1] : 0.0;
  }
  HIP_TRY(ctx, hipMemcpyAsync(d_offs, offsets, (size_t)(n_cfg + 1) * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
  if (nops > 0) {
    HIP_TRY(ctx, hipMemcpyAsync(d_tau, tau, (size_t)nops * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d_op, op, (size_t)nops * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  }
  HIP_TRY(ctx, hipMemcpyAsync(d_w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_wlog, wlog.data(), wlog.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_weight, wt.data(), wt.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(d_roff, roff.data(), roff.size() * sizeof(long long), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync(d_rho, 0, (size_t)entries * 2 * sizeof(double), ctx->stream));
  a.offsets = d_offs;
  a.tau = d_tau;
  a.op = d_op;
  a.log_thr = nullptr;
  a.out = nullptr;
  a.panel = ctr::kPanel;
  hipError_t e = ctr::launch_plan(ctx->imp, a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "plan kernel");
  if ((e = ctr::launch_scan(a, ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "scan kernel");
  ctr::RdmArgs r{};
  r.buf = d_buf;
  r.per_wg = per_wg;
  r.slots = slots;
  r.w = d_w;
  r.wlog = d_wlog;
  r.weight = d_weight;
  r.rho = d_rho;
  r.rho_off = d_roff;
  if ((e = ctr::launch_rdm(ctx->imp, a, r, grid, ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "density-matrix kernel");
  HIP_TRY(ctx, hipMemcpyAsync(rho, d_rho, (size_t)entries * 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CTR_OK;
}

ctr_status ctr_bound(ctr_ctx* ctx, int32_t n_ops, const double* tau, const int32_t* op, double* log_bound) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  if (!log_bound || n_ops < 0) return fail(ctx, CTR_ERR_ARG, "bad argument");
  const int64_t offs[2] = {0, n_ops};
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, nullptr, &split, &kind)) != CTR_OK) return s;
  return host_batch(ctx, 1, offs, tau, op, nullptr, nullptr, log_bound, 1, false, kind);
}

ctr_status ctr_strings(ctr_ctx* ctx, int32_t n_ops, const int32_t* op, int32_t* q0_out, int32_t* n_out) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  if (!q0_out || !n_out || n_ops < 0 || (n_ops > 0 && !op)) return fail(ctx, CTR_ERR_ARG, "bad argument");
  std::vector<double> tau((size_t)std::max(n_ops, 1), 0.0);
  const int64_t offs[2] = {0, n_ops};
  double lb = 0.0;
  BatchArgs a{};
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, nullptr, &split, &kind)) != CTR_OK) return s;
  if ((s = host_batch(ctx, 1, offs, tau.data(), op, nullptr, nullptr, &lb, 1, false, kind, &a)) != CTR_OK) return s;
  std::vector<StrRec> rec(ctx->n_sec);
  HIP_TRY(ctx, hipMemcpyAsync(rec.data(), a.rec, rec.size() * sizeof(StrRec), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  int k = 0;
  for (int q = 0; q < ctx->n_sec; ++q)
    if (rec[q].n_panels > 0) q0_out[k++] = q;
  *n_out = k;
  return CTR_OK;
}

ctr_status ctr_trace_batch_device(ctr_ctx* ctx, int32_t n_cfg, const int64_t* d_offsets, const double* d_tau,
                                  const int32_t* d_op, const ctr_opts* opts, ctr_value* d_out) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, opts, &split, &kind, n_cfg)) != CTR_OK) return s;
  const bool auto_kind = !opts || opts->kernel == CTR_KERNEL_AUTO;
  if (n_cfg < 0 || (n_cfg > 0 && (!d_offsets || !d_out))) return fail(ctx, CTR_ERR_ARG, "null argument");
  const size_t free_bytes = ctx->arena_bytes - ctx->resident;
  const size_t per_cfg = scratch_per_cfg(ctx) + 64;
  const long long fit = (long long)((free_bytes > 8 * kAlign ? free_bytes - 8 * kAlign : 0) / per_cfg);
  if (n_cfg > 0 && fit < 1) return fail(ctx, CTR_ERR_OOM, "arena too small for one configuration");
  long long cap = fit;  // chunk cap, halved while the grouped rounds do not fit
  for (int32_t c0 = 0; c0 < n_cfg;) {
    const int32_t m = (int32_t)std::min<long long>(cap, n_cfg - c0);
    Bump b{ctx->arena, ctx->resident, ctx->arena_bytes};
    BatchArgs a{};
    if (!carve(ctx, b, m, a)) return fail(ctx, CTR_ERR_OOM, "arena too small");
    a.offsets = (const long long*)d_offsets + c0;
    a.tau = d_tau;
    a.op = d_op;
    a.log_thr = nullptr;
    a.out = d_out + c0;
    s = enqueue(ctx, a, false, split, kind, &b);
    if (s == CTR_ERR_OOM && kind == Kernel::Group) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      if (m > 1) {
        cap = m / 2;
      } else if (auto_kind) {
        kind = per_string_kernel(ctx);
        cap = fit;
      } else {
        return s;
      }
      ctx->err.clear();
      continue;
    }
    if (s != CTR_OK) return s;
    c0 += m;
  }
  return CTR_OK;
}

ctr_status ctr_trace_batch_device_static(ctr_ctx* ctx, int32_t n_cfg, const int64_t* d_offsets, const double* d_tau,
                                         const int32_t* d_op, const ctr_opts* opts, ctr_value* d_out) {
  ctr_status s = ready(ctx);
  if (s != CTR_OK) return s;
  bool split = false;
  Kernel kind = Kernel::Block;
  if ((s = check_opts(ctx, opts, &split, &kind, n_cfg)) != CTR_OK) return s;
  if (kind == Kernel::Group) {
    // the grouped rounds size their scratch from a device count read back mid-call
    if (opts && (opts->kernel == CTR_KERNEL_GROUPED || opts->kernel == CTR_KERNEL_GROUPED_ROWS))
      return fail(ctx, CTR_ERR_UNSUPPORTED, "the static-scratch entry point runs the per-string kernels only");
    kind = per_string_kernel(ctx);
  }
  if (n_cfg < 0 || (n_cfg > 0 && (!d_offsets || !d_out))) return fail(ctx, CTR_ERR_ARG, "null argument");
  if (n_cfg == 0) return CTR_OK;
  void* base = g_scratch[ctx->device];
  if (!base) return fail(ctx, CTR_ERR_STATE, "static scratch address not set up for this device");
  Bump b{(char*)base, 0, kStaticScratchBytes};
  BatchArgs a{};
  if (!carve(ctx, b, n_cfg, a)) {
    Bump probe{(char*)kAlign, 0, SIZE_MAX / 2};  // sizes only, never dereferenced
    BatchArgs t{};
    carve(ctx, probe, n_cfg, t);
    return fail(ctx, CTR_ERR_OOM, "batch needs " + std::to_string(probe.off >> 10) + " KiB of per-call scratch; the "
                                      "static array holds " + std::to_string(kStaticScratchBytes >> 10) + " KiB");
  }
  a.offsets = (const long long*)d_offsets;
  a.tau = d_tau;
  a.op = d_op;
  a.log_thr = nullptr;
  a.out = d_out;
  // no events either: this call creates nothing
  const bool timing = ctx->timing;
  ctx->timing = false;
  s = enqueue(ctx, a, false, split, kind, nullptr);
  ctx->timing = timing;
  return s;
}

ctr_status ctr_probe_peaks(ctr_ctx* ctx, double* out) {
  if (!ctx || !out) return CTR_ERR_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  ctx->err.clear();
  const size_t off = align_up(ctx->resident);
  if (off + 256 * sizeof(double) > ctx->arena_bytes) return fail(ctx, CTR_ERR_OOM, "arena too small for the probe");
  const hipError_t e = ctr::probe_peaks(ctx->device, ctx->stream, (double*)(ctx->arena + off), out);
  if (e != hipSuccess) return hip_fail(ctx, e, "peak probe");
  return CTR_OK;
}

ctr_status ctr_kernel_timing(ctr_ctx* ctx, int32_t on) {
  if (!ctx) return CTR_ERR_ARG;
  ctx->timing = on != 0;
  return CTR_OK;
}

ctr_status ctr_kernel_timing_read(ctr_ctx* ctx, double* total_ms, int32_t* n_launches) {
  if (!ctx || !total_ms || !n_launches) return CTR_ERR_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double sum = 0.0;
  for (auto& ev : ctx->events) {
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ev.first, ev.second));
    sum += ms;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  *total_ms = sum;
  *n_launches = (int32_t)ctx->events.size();
  ctx->events.clear();
  return CTR_OK;
}

ctr_status ctr_last_kernel(const ctr_ctx* ctx, int32_t* kernel, int32_t* slices) {
  if (!ctx || !kernel) return CTR_ERR_ARG;
  *kernel = ctx->last_kernel;
  if (slices) *slices = ctx->last_slices;
  return CTR_OK;
}

ctr_status ctr_synchronize(ctr_ctx* ctx) {
  if (!ctx) return CTR_ERR_ARG;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return CTR_OK;
}

}  // extern "C"
