// C ABI of libmosaic: argument validation, workspace layout, and the
// host-side drivers of the sweep (Alg. 2 on one device).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "mf_internal.h"

namespace mf {

static thread_local char g_err[512] = "";

mf_status fail(mf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

static mf_status ok() {
  g_err[0] = '\0';
  return MF_OK;
}

NetLayout net_layout(int width, int prec, size_t base, int n_in) {
  NetLayout L;
  L.width = width;
  L.prec = prec;
  const size_t d = (size_t)width;
  size_t o = align256(base);
  L.w1gT = o; o = align256(o + (size_t)n_in * d * 4);
  L.w1gb = o; if (prec != MF_FP32 && n_in == 128) o = align256(o + 128 * d * 2);
  L.w1x = o;  o = align256(o + 2 * d * 4);
  L.b1 = o;   o = align256(o + d * 4);
  L.wh = o;   o = align256(o + 3 * d * d * (prec == MF_FP32 ? 4 : 2));
  L.bh = o;   o = align256(o + 3 * d * 4);
  L.w5 = o;   o = align256(o + d * 4);
  L.b5 = o;   o = align256(o + 8);
  L.end = o;
  return L;
}

NetPtrs net_ptrs(const NetLayout& L, const void* ws) {
  const char* b = static_cast<const char*>(ws);
  NetPtrs p;
  p.w1gT = reinterpret_cast<const float*>(b + L.w1gT);
  p.w1gb = static_cast<const void*>(b + L.w1gb);
  p.w1x = reinterpret_cast<const float*>(b + L.w1x);
  p.b1 = reinterpret_cast<const float*>(b + L.b1);
  p.wh = static_cast<const void*>(b + L.wh);
  p.bh = reinterpret_cast<const float*>(b + L.bh);
  p.w5 = reinterpret_cast<const float*>(b + L.w5);
  p.b5 = reinterpret_cast<const float*>(b + L.b5);
  return p;
}

SweepLayout sweep_layout(int width, int prec, const mf_domain_desc* dom, int n_domains, int mode, int embed_c) {
  SweepLayout S;
  S.net = net_layout(width, prec, 0, embed_c ? embed_c * 128 : 128);
  size_t o = S.net.end;
  int64_t n_skel = 0;
  for (int d = 0; d < n_domains; ++d) n_skel += skeleton_count(dom[d].units_x, dom[d].units_y);
  S.skel = o; o = align256(o + (size_t)n_skel * 4);
  S.part = o; o = align256(o + 2 * (size_t)kDeltaBlocks * n_domains * 4);
  S.dres = o; o = align256(o + 2 * (size_t)n_domains * 4);
  S.table = o;
  o = align256(o + (size_t)n_domains * sizeof(DomEntry) + 2 * 4 * ((size_t)n_domains + 1) * 4);
  int64_t span = 0;
  for (int d = 0; d < n_domains; ++d)
    span = std::max<int64_t>(span, dom[d].field_offset + (32LL * dom[d].units_y) * dom[d].pitch +
                                       32LL * dom[d].units_x + 1);
  S.anext = o;   // the additive mode's next field; the multiplicative mode needs none
  if (mode == MF_ADDITIVE) o = align256(o + (size_t)span * 4);
  if (embed_c) {   // the GELU network's phase chunks: projections, target coordinates, two row buffers
    S.gC = o; o = align256(o + (size_t)(kGeluRows / 61) * width * 4);
    S.gX = o; o = align256(o + (61 + 961) * 2 * 4);
    for (int l = 0; l < 2; ++l) { S.gZ[l] = o; o = align256(o + (size_t)kGeluRows * width * 4); }
  }
  S.total = o;
  return S;
}

TrainLayout train_layout(const mf_sdnet_desc* desc, int64_t B, int64_t nd, int64_t nc) {
  TrainLayout T;
  const int width = desc->width;
  const bool gelu = desc->activation == MF_GELU;
  const int C = gelu ? desc->embed_channels : 0;
  T.net = net_layout(width, MF_FP32, 0, gelu ? 128 * C : 128);
  const size_t d = (size_t)width;
  const size_t SR = (size_t)std::max<int64_t>(4 * B * nc, B * nd);   // stream rows
  const size_t chunks = kBwdGroups;   // weight-gradient partials: one per reverse-kernel workgroup
  const size_t P = (size_t)mf_param_count(desc);
  size_t o = T.net.end;
  T.whT = o; o = align256(o + 3 * d * d * 4);
  T.C = o;   o = align256(o + (size_t)B * d * 4);
  for (int l = 0; l < 4; ++l) { T.Z[l] = o; o = align256(o + SR * d * 4); }
  // tanh: Sv[0] (layer 1) is never stored, its a_x, a_y, a_L being W1x and 0
  // for every row; GELU keeps layer 1's pre-activations there
  for (int l = gelu ? 0 : 1; l < 4; ++l) { T.Sv[l] = o; o = align256(o + SR * d * 4); }
  for (int l = 0; l < 2; ++l) { T.Ab[l] = o; o = align256(o + SR * d * 4); }
  const size_t l1parts = (size_t)kL1MaxChunks * d * ((gelu ? 128 * C : 128) + 3);
  T.wpart = o; o = align256(o + std::max(chunks * d * d, l1parts) * 4);
  T.bpart = o; o = align256(o + chunks * d * 4);
  for (int l = 0; l < 2; ++l) { T.opart[l] = o; o = align256(o + (size_t)kOutWaves * (d + 2) * 4); }
  for (int l = 0; l < 2; ++l) { T.l1[l] = o; o = align256(o + 3 * (size_t)B * d * 4); }
  T.grad = o; o = align256(o + P * 4);
  if (gelu) {
    T.emb = o;   o = align256(o + (size_t)B * 128 * C * 4);
    T.cpart = o; o = align256(o + (size_t)B * embed_param_offset(C) * 4);
  }
  T.total = o;
  return T;
}

TrainBuffers train_buffers(const TrainLayout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  TrainBuffers t;
  t.C = reinterpret_cast<float*>(b + L.C);
  for (int l = 0; l < 4; ++l) {
    t.Z[l] = reinterpret_cast<float*>(b + L.Z[l]);
    t.Sv[l] = L.Sv[l] == 0 ? nullptr : reinterpret_cast<float*>(b + L.Sv[l]);
  }
  for (int l = 0; l < 2; ++l) {
    t.Ab[l] = reinterpret_cast<float*>(b + L.Ab[l]);
    t.opart[l] = reinterpret_cast<float*>(b + L.opart[l]);
    t.l1[l] = reinterpret_cast<float*>(b + L.l1[l]);
  }
  t.wpart = reinterpret_cast<float*>(b + L.wpart);
  t.bpart = reinterpret_cast<float*>(b + L.bpart);
  t.grad = reinterpret_cast<float*>(b + L.grad);
  t.emb = L.emb ? reinterpret_cast<float*>(b + L.emb) : nullptr;
  t.cpart = L.cpart ? reinterpret_cast<float*>(b + L.cpart) : nullptr;
  return t;
}

#define MF_TRY(expr)                 \
  do {                               \
    mf_status _s = (expr);           \
    if (_s != MF_OK) return _s;      \
  } while (0)

#define MF_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return fail(MF_EDEVICE, "%s: %s", #expr, hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static mf_status check_desc(const mf_sdnet_desc* d) {
  if (!d) return fail(MF_EINVAL, "sdnet descriptor is NULL");
  if (d->width != 128 && d->width != 256)
    return fail(MF_ESHAPE, "sdnet width %d unsupported (128 or 256)", d->width);
  if (d->depth != 4) return fail(MF_ESHAPE, "sdnet depth %d unsupported (4)", d->depth);
  if (d->n_boundary != 128)
    return fail(MF_ESHAPE, "n_boundary %d unsupported (128)", d->n_boundary);
  if (d->activation == MF_TANH) {
    if (d->embed_channels != 0)
      return fail(MF_ESHAPE, "the tanh network has no boundary embedding (embed_channels %d, must be 0)",
                  d->embed_channels);
  } else if (d->activation == MF_GELU) {
    if (d->embed_channels < 1 || d->embed_channels > 8)
      return fail(MF_ESHAPE, "embed_channels %d not in 1..8 for the GELU network", d->embed_channels);
  } else {
    return fail(MF_EINVAL, "activation %d unknown", d->activation);
  }
  return MF_OK;
}

static bool is_gelu(const mf_sdnet_desc* d) { return d->activation == MF_GELU; }

// The entry points built for the tanh network only.
static mf_status need_tanh(const mf_sdnet_desc* d, const char* what) {
  if (is_gelu(d)) return fail(MF_EUNSUPPORTED, "%s is built for the tanh network only", what);
  return MF_OK;
}

// The GELU network runs in float32, multiplicative sweeps.
static mf_status gelu_limits(const mf_sdnet_desc* d, int prec, int mode) {
  if (!is_gelu(d)) return MF_OK;
  if (prec != MF_FP32) return fail(MF_EUNSUPPORTED, "the GELU network runs in MF_FP32 only");
  if (mode != MF_MULTIPLICATIVE) return fail(MF_EUNSUPPORTED, "the GELU network runs multiplicative sweeps only");
  return MF_OK;
}

static bool valid_tile_rows(int prec, int rows) {
  if (prec == MF_FP32) return rows == 32 || rows == 64 || rows == (64 | MF_TILE_STREAM);
  if (rows & MF_TILE_STREAM) return false;
  if (prec == MF_FP16 && (rows & MF_TILE_WIDE)) return false;
  if (rows & MF_TILE_ROWSPLIT)
    return (rows & ~MF_TILE_PERSIST) == (256 | MF_TILE_ROWSPLIT) || (rows & ~MF_TILE_PERSIST) == (128 | MF_TILE_ROWSPLIT);
  const int r = rows & ~MF_TILE_WIDE;
  if (rows & MF_TILE_WIDE) return r == 128 || r == 256;
  return r == 64 || r == 128 || r == 256;
}

static mf_status check_prec(int prec) {
  if (prec != MF_FP32 && prec != MF_BF16 && prec != MF_FP16) return fail(MF_EINVAL, "precision %d unknown", prec);
  return MF_OK;
}

static mf_status check_one_domain(const mf_domain_desc* dom, int d) {
  if (dom->units_x < 1 || dom->units_y < 1)
    return fail(MF_ESHAPE, "domain %d: units %d x %d: each must be >= 1", d, dom->units_x, dom->units_y);
  if (dom->units_x > 4096 || dom->units_y > 4096)
    return fail(MF_ESHAPE, "domain %d: units %d x %d exceed 4096", d, dom->units_x, dom->units_y);
  if (dom->cells_per_unit != 32) return fail(MF_ESHAPE, "domain %d: cells_per_unit must be 32", d);
  if (dom->stride != 16) return fail(MF_ESHAPE, "domain %d: placement stride must be 16 cells", d);
  const int64_t nx = 32LL * dom->units_x + 1, ny = 32LL * dom->units_y + 1;
  if (dom->pitch < nx)
    return fail(MF_ESHAPE, "domain %d: pitch %lld < row length %lld", d, (long long)dom->pitch, (long long)nx);
  if (dom->field_offset < 0) return fail(MF_ESHAPE, "domain %d: field_offset must be >= 0", d);
  if ((ny - 1) * dom->pitch + nx > (1LL << 40)) return fail(MF_ESHAPE, "domain %d: field too large", d);
  return MF_OK;
}

// One domain, or a batch of 2..4096 independent domains in one packed
// buffer whose element ranges must not overlap (their phases run
// concurrently).
// Floats from a domain's first element to one past its last grid point.
static int64_t field_extent(const mf_domain_desc& d) {
  return (32LL * d.units_y) * d.pitch + 32LL * d.units_x + 1;
}

static mf_status check_domain(const mf_domain_desc* dom, int n_domains) {
  if (!dom) return fail(MF_EINVAL, "domain descriptor is NULL");
  if (n_domains < 1 || n_domains > 4096)
    return fail(MF_ESHAPE, "n_domains = %d not in 1..4096", n_domains);
  std::vector<std::pair<int64_t, int64_t>> ext;
  for (int d = 0; d < n_domains; ++d) {
    MF_TRY(check_one_domain(&dom[d], d));
    const int64_t nx = 32LL * dom[d].units_x + 1, ny = 32LL * dom[d].units_y + 1;
    ext.emplace_back(dom[d].field_offset, dom[d].field_offset + (ny - 1) * dom[d].pitch + nx);
  }
  std::sort(ext.begin(), ext.end());
  for (size_t i = 1; i < ext.size(); ++i)
    if (ext[i].first < ext[i - 1].second) return fail(MF_EINVAL, "domains overlap in the field buffer");
  return MF_OK;
}

static mf_status check_ptr(const void* p, const char* name, size_t align = 4) {
  if (!p) return fail(MF_EINVAL, "%s is NULL", name);
  if (!aligned(p, align)) return fail(MF_EINVAL, "%s is not %zu-byte aligned", name, align);
  return MF_OK;
}

static mf_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return MF_OK;
  if (!ws) return fail(MF_EINVAL, "workspace is NULL (%zu bytes needed)", need);
  if (!aligned(ws, 256)) return fail(MF_EINVAL, "workspace is not 256-byte aligned");
  if (ws_bytes < need) return fail(MF_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  return MF_OK;
}

// Static device scratch of mf_sweep_noalloc: the prepared network and the
// batch table of one call, for callers that cannot allocate a workspace.
// Each device holds its own copy for the life of the process; host code
// never uses the array's name as an address, only the per-device pointer
// taken with hipGetSymbolAddress when a context is created on that device.
constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Address of this device's scratch array (the device must be current).
static mf_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(MF_EDEVICE, "device %d: static scratch is kept for devices 0..%d", device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return MF_OK;
}

// Layout of the no-alloc sweep inside the static scratch: the prepared
// network, then the batch table. Multiplicative sweeps evaluate no delta
// and keep no next field, so nothing else is needed.
static SweepLayout noalloc_layout(int width, int prec, int n_domains) {
  SweepLayout S;
  S.net = net_layout(width, prec, 0);
  S.table = S.net.end;
  const size_t end =
      align256(S.table + (size_t)n_domains * sizeof(DomEntry) + 2 * 4 * ((size_t)n_domains + 1) * 4);
  S.skel = S.part = S.dres = S.anext = end;
  S.total = end;
  return S;
}

}  // namespace mf

using namespace mf;

// A captured run of `sweeps` consecutive sweeps (4 colour-phase launches
// each) for one field / workspace / network configuration.
struct SweepGraph {
  const float* field;
  const void* ws;
  int64_t pitch;
  int ux, uy, width, prec, targets, mode, sweeps;
  uint64_t key;
  hipGraphExec_t exec;
};

// Tile height chosen by mf_autotune for one phase configuration: a single
// domain (by its units) or a batch (by the hash of its descriptors).
struct TuneEntry {
  int width, prec, targets, ux, uy, rows;
  uint64_t key;   // batches: domain-list hash; single domains: 0
};

struct mf_ctx {
  int device;
  int n_cu;
  void* scratch = nullptr;            // this device's static scratch (mf_sweep_noalloc)
  int force_rows[3] = {0, 0, 0};      // per precision; 0 = automatic
  std::vector<TuneEntry> tuned;
  hipStream_t gstream = nullptr;     // graph launches (default priority)
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<SweepGraph> graphs;
  bool use_graphs = true;
  bool timing = false;
  std::vector<hipEvent_t> events;   // pairs (start, stop) of timed launches
  std::vector<int64_t> rows;        // point evaluations of each timed record
  std::vector<int64_t> nlaunch;     // colour-phase launches in each timed record
  size_t used = 0;                  // pairs recorded since the last read
  int fault_sweep = 0, fault_colour = 0;   // MF_FAULT_INJECT: fail before this phase (0 = off)
};

// MF_FAULT_INJECT=k:c makes mf_solve fail with MF_EDEVICE just before colour
// phase c (0..3) of sweep k (>= 1) of a multiplicative solve, leaving the
// field as the earlier phases made it. Parsed once per context; anything
// else leaves injection off.
static void parse_fault_inject(const char* v, int* sweep, int* colour) {
  *sweep = 0;
  *colour = 0;
  int k = 0, c = 0;
  char tail = 0;
  if (v && sscanf(v, "%d:%d%c", &k, &c, &tail) == 2 && k >= 1 && c >= 0 && c <= 3) {
    *sweep = k;
    *colour = c;
  }
}

extern "C" {

const char* mf_last_error(void) { return g_err; }

int32_t mf_fault_inject_parse(const char* spec, int32_t* sweep, int32_t* colour) {
  int k, c;
  parse_fault_inject(spec, &k, &c);
  if (sweep) *sweep = k;
  if (colour) *colour = c;
  return k > 0 ? 1 : 0;
}

int64_t mf_param_count(const mf_sdnet_desc* desc) {
  if (check_desc(desc) != MF_OK) return -1;
  const int64_t d = desc->width;
  if (is_gelu(desc)) {
    const int64_t C = desc->embed_channels;
    return embed_param_offset((int)C) + d * (C * desc->n_boundary + 2) + d + 3 * (d * d + d) + d + 1;
  }
  return d * (desc->n_boundary + 2) + d + 3 * (d * d + d) + d + 1;
}

mf_status mf_ctx_create(int device, mf_ctx** out) {
  if (!out) return fail(MF_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(MF_EDEVICE, "no GPU available (%s)", e == hipSuccess ? "0 devices" : hipGetErrorString(e));
  if (device < 0 || device >= n) return fail(MF_EDEVICE, "device %d out of range [0, %d)", device, n);
  hipDeviceProp_t prop;
  MF_HIP(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MF_EDEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  MF_HIP(hipSetDevice(device));
  mf_ctx* c = new (std::nothrow) mf_ctx;
  if (!c) return fail(MF_ENOMEM, "host allocation failed");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  parse_fault_inject(getenv("MF_FAULT_INJECT"), &c->fault_sweep, &c->fault_colour);
  {
    const mf_status st = scratch_address(device, &c->scratch);
    if (st != MF_OK) {
      delete c;
      return st;
    }
  }
  if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess) {
    mf_ctx_destroy(c);
    return fail(MF_EDEVICE, "stream/event creation failed");
  }
  *out = c;
  return ok();
}

void mf_ctx_destroy(mf_ctx* ctx) {
  if (!ctx) return;
  for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
  for (SweepGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->join) (void)hipEventDestroy(ctx->join);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  delete ctx;
}

mf_status mf_ctx_tile_rows(mf_ctx* ctx, int32_t prec, int32_t rows) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_TRY(check_prec(prec));
  if (rows != 0 && !valid_tile_rows(prec, rows))
    return fail(MF_EINVAL, "tile rows %d not available for precision %d", rows, prec);
  ctx->force_rows[prec] = rows;
  for (SweepGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);   // captured shapes change
  ctx->graphs.clear();
  return ok();
}

mf_status mf_ctx_graphs(mf_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  ctx->use_graphs = enable != 0;
  return ok();
}

mf_status mf_ctx_timing(mf_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  ctx->timing = enable != 0;
  return ok();
}

mf_status mf_ctx_timing_read(mf_ctx* ctx, int64_t* launches, double* total_ms, int64_t* rows) {
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  double ms = 0.0;
  int64_t nrows = 0, nl = 0;
  for (size_t i = 0; i < ctx->used; ++i) {
    MF_HIP(hipEventSynchronize(ctx->events[2 * i + 1]));
    float t = 0.0f;
    MF_HIP(hipEventElapsedTime(&t, ctx->events[2 * i], ctx->events[2 * i + 1]));
    ms += t;
    nrows += ctx->rows[i];
    nl += ctx->nlaunch[i];
  }
  if (launches) *launches = nl;
  if (total_ms) *total_ms = ms;
  if (rows) *rows = nrows;
  ctx->used = 0;
  return ok();
}

mf_status mf_workspace_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                            int32_t prec, int32_t targets, int32_t mode, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  MF_TRY(check_domain(dom, n_domains));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (mode != MF_MULTIPLICATIVE && mode != MF_ADDITIVE) return fail(MF_EINVAL, "mode %d unknown", mode);
  MF_TRY(gelu_limits(desc, prec, mode));
  *bytes = sweep_layout(desc->width, prec, dom, n_domains, mode, desc->embed_channels).total;
  return ok();
}

static mf_status sweep_common_checks(const mf_sdnet_desc* desc, const float* params, float* u,
                                     const mf_domain_desc* dom, int32_t n_domains, int32_t targets,
                                     int32_t mode, int32_t prec, void* ws, size_t ws_bytes,
                                     SweepLayout* L) {
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  MF_TRY(check_domain(dom, n_domains));
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(u, "u"));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (mode != MF_MULTIPLICATIVE && mode != MF_ADDITIVE) return fail(MF_EINVAL, "mode %d unknown", mode);
  MF_TRY(gelu_limits(desc, prec, mode));
  *L = sweep_layout(desc->width, prec, dom, n_domains, mode, desc->embed_channels);
  MF_TRY(check_ws(ws, ws_bytes, L->total));
  return MF_OK;
}

static mf_status timing_begin(mf_ctx* ctx, hipStream_t s) {
  if (ctx->events.size() < 2 * (ctx->used + 1)) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      MF_HIP(hipEventCreate(&e));
      ctx->events.push_back(e);
    }
    ctx->rows.push_back(0);
    ctx->nlaunch.push_back(0);
  }
  MF_HIP(hipEventRecord(ctx->events[2 * ctx->used], s));
  return MF_OK;
}

static mf_status timing_end(mf_ctx* ctx, hipStream_t s, int64_t rows, int64_t launches) {
  MF_HIP(hipEventRecord(ctx->events[2 * ctx->used + 1], s));
  ctx->rows[ctx->used] = rows;
  ctx->nlaunch[ctx->used] = launches;
  ctx->used++;
  return MF_OK;
}

static int64_t phase_rows(const mf_domain_desc* dom, int colour, int targets) {
  const int64_t n_place = (int64_t)(dom->units_x - (colour & 1)) * (dom->units_y - (colour >> 1));
  return n_place * (targets == MF_INTERIOR ? 961 : 61);
}

// Everything a colour phase needs: one domain, or a batch whose domain table
// and per-colour tile prefixes were uploaded into the workspace.
struct Plan {
  int nd = 1;
  const mf_domain_desc* dom = nullptr;   // host descriptors
  float* u = nullptr;                    // caller's buffer (offsets are relative to it)
  int width = 0, prec = 0, targets = 0, mode = MF_MULTIPLICATIVE;
  NetPtrs net{};
  const void* ws = nullptr;
  float* anext = nullptr;                         // additive: the next field
  const DomEntry* d_doms = nullptr;
  const int32_t* d_tb[2] = {nullptr, nullptr};   // [4][nd + 1]: sweep targets, assembly
  int R[2] = {0, 0};                              // tile rows (batched)
  int64_t n_tiles[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  int64_t rows[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  uint64_t key = 0;                               // identifies the domain list
  // the GELU network (activation MF_GELU): unfused phases in row chunks
  int embed_c = 0;                                // embedding channels; 0 = the tanh tile kernels
  const float* params = nullptr;                  // caller's flat parameters (convolutions)
  float* gC = nullptr;                            // [chunk placements][d] projections
  float* gX[2] = {nullptr, nullptr};              // target coordinates: CROSS, INTERIOR
  float* gZ[2] = {nullptr, nullptr};              // [kGeluRows][d] value rows
};

static int tile_rows_for(const mf_ctx* ctx, int width, int prec, int targets, const mf_domain_desc* dom,
                         int nd, int64_t rows, uint64_t key = 0) {
  if (ctx->force_rows[prec]) return ctx->force_rows[prec];
  for (const TuneEntry& t : ctx->tuned)
    if (t.width == width && t.prec == prec && t.targets == targets &&
        (nd == 1 ? (t.key == 0 && t.ux == dom->units_x && t.uy == dom->units_y) : t.key == key))
      return t.rows;
  const int64_t n_cu = ctx->n_cu;
  // bf16 and fp16: the 256-row row-split tile from half such a tile per CU up
  // (32 x 32 units, ~0.9 tiles per CU: 32.5 against 42.4 us per phase with
  // 64-row tiles; 24 x 24 units, ~0.5: 30.5 against 31.2 us); below that the
  // 64-row column-split tile spreads the rows over more CUs (16 x 16 units:
  // 17.6 against 30.1 us)
  if (prec != MF_FP32) return rows >= 128 * n_cu ? (256 | MF_TILE_ROWSPLIT) : 64;
  // fp32: 64-row tiles with register weights from one 32-row tile per CU up
  // (a 16 x 16-unit phase, ~0.9 such tiles per CU: 54 us against 61 us with
  // 32-row tiles); below that, 32-row tiles spread the few rows over more CUs.
  // From two 64-row tiles per CU up a single domain streams the weights
  // instead (64 x 64 units: 804 against 818 us per sweep phase, 12.07 against
  // 12.24 ms per assembly phase); the batched kernel's streamed form spills.
  if (rows < 32 * n_cu) return 32;
  return nd == 1 && rows >= 128 * n_cu ? (64 | MF_TILE_STREAM) : 64;
}

static mf_status make_plan(mf_ctx* ctx, const mf_sdnet_desc* desc, int prec, int targets, int mode,
                           float* u, const mf_domain_desc* dom, int nd, void* ws, const SweepLayout& L,
                           hipStream_t s, Plan* P) {
  P->nd = nd;
  P->mode = mode;
  P->anext = reinterpret_cast<float*>(static_cast<char*>(ws) + L.anext);
  P->dom = dom;
  P->u = u;
  P->width = desc->width;
  P->prec = prec;
  P->targets = targets;
  P->net = net_ptrs(L.net, ws);
  P->ws = ws;
  P->embed_c = desc->embed_channels;
  if (P->embed_c) {
    char* b = static_cast<char*>(ws);
    P->gC = reinterpret_cast<float*>(b + L.gC);
    P->gX[0] = reinterpret_cast<float*>(b + L.gX);
    P->gX[1] = P->gX[0] + 61 * 2;
    P->gZ[0] = reinterpret_cast<float*>(b + L.gZ[0]);
    P->gZ[1] = reinterpret_cast<float*>(b + L.gZ[1]);
    MF_HIP(launch_target_coords(P->gX[0], P->gX[1], s));
  }
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 4; ++c)
      for (int d = 0; d < nd; ++d) P->rows[a][c] += phase_rows(&dom[d], c, a ? MF_INTERIOR : targets);
  uint64_t h = 1469598103934665603ull;                  // FNV-1a over the descriptors
  const unsigned char* bytes = reinterpret_cast<const unsigned char*>(dom);
  for (size_t i = 0; i < (size_t)nd * sizeof(mf_domain_desc); ++i) h = (h ^ bytes[i]) * 1099511628211ull;
  P->key = h;
  if (nd == 1) return MF_OK;
  std::vector<char> host((size_t)nd * sizeof(DomEntry) + 2 * 4 * ((size_t)nd + 1) * 4);
  DomEntry* he = reinterpret_cast<DomEntry*>(host.data());
  int32_t* htb = reinterpret_cast<int32_t*>(host.data() + (size_t)nd * sizeof(DomEntry));
  for (int d = 0; d < nd; ++d)
    he[d] = DomEntry{dom[d].field_offset, dom[d].pitch, dom[d].units_x, dom[d].units_y};
  for (int a = 0; a < 2; ++a) {
    const int tg = a ? MF_INTERIOR : targets;
    P->R[a] = tile_rows_for(ctx, desc->width, prec, tg, dom, nd, P->rows[a][0], h);
    for (int c = 0; c < 4; ++c) {
      int32_t* tb = htb + (a * 4 + c) * (nd + 1);
      int64_t acc = 0;
      for (int d = 0; d < nd; ++d) {
        tb[d] = (int32_t)acc;
        const int rows_per_tile = P->R[a] & 0xffff;
        acc += (phase_rows(&dom[d], c, tg) + rows_per_tile - 1) / rows_per_tile;
      }
      if (acc > INT32_MAX) return fail(MF_ESHAPE, "batch has too many tiles");
      tb[nd] = (int32_t)acc;
      P->n_tiles[a][c] = acc;
    }
  }
  char* dst = static_cast<char*>(ws) + L.table;
  MF_HIP(hipMemcpyAsync(dst, host.data(), host.size(), hipMemcpyHostToDevice, s));
  P->d_doms = reinterpret_cast<const DomEntry*>(dst);
  P->d_tb[0] = reinterpret_cast<const int32_t*>(dst + (size_t)nd * sizeof(DomEntry));
  P->d_tb[1] = P->d_tb[0] + 4 * (nd + 1);
  return MF_OK;
}

// One colour phase of the plan:
//   PH_SWEEP     predictions stored into u at the plan's targets;
//   PH_ASSEMBLY  INTERIOR predictions / cover count accumulated into out;
//   PH_ADDITIVE  predictions at the plan's targets / cover count accumulated into out.
// Sweep and additive phases are timed when the context's timing is on.
enum { PH_SWEEP = 0, PH_ASSEMBLY = 1, PH_ADDITIVE = 2 };
// A colour phase of the GELU network, domain by domain, in chunks of at most
// kGeluRows rows: embedding + projection per placement (gathered from the
// field), the value stream through the four GELU layers, and the output
// layer storing at the targets (sweep) or averaging into out (assembly).
// Chunks of one colour may run in any order: same-colour placements never
// read each other's targets.
static mf_status run_colour_gelu(const Plan& P, int colour, int kind, float* out, hipStream_t s) {
  const int tg = kind == PH_ASSEMBLY ? MF_INTERIOR : P.targets;
  const int T = tg == MF_INTERIOR ? 961 : 61;
  const int chunk = (int)(kGeluRows / T);
  float* Z[4] = {P.gZ[0], P.gZ[1], P.gZ[0], P.gZ[1]};
  for (int d = 0; d < P.nd; ++d) {
    const mf_domain_desc& D = P.dom[d];
    const int n_q = (D.units_x - (colour & 1)) * (D.units_y - (colour >> 1));
    const float* u = P.u + D.field_offset;
    float* dst = (kind == PH_SWEEP ? P.u : out) + D.field_offset;
    for (int q0 = 0; q0 < n_q; q0 += chunk) {
      const int nq = std::min(chunk, n_q - q0);
      MF_HIP(launch_embed_project(P.params, P.width, P.embed_c, P.net, nullptr, nq, u, D.pitch, D.units_x, colour,
                                  q0, P.gC, s));
      MF_HIP(launch_value_forward_act(P.net, P.width, ACT_GELU, P.gC, P.gX[tg], 0, T, (int64_t)nq * T, Z, s));
      MF_HIP(launch_rows_output(P.net, P.width, tg, Z[3], (int64_t)nq * T, kind == PH_SWEEP ? 1 : 2, dst, D.pitch,
                                D.units_x, D.units_y, colour, q0, s));
    }
  }
  return MF_OK;
}

static mf_status run_colour(mf_ctx* ctx, const Plan& P, int colour, int kind, float* out, hipStream_t s,
                            bool allow_timing = true) {
  const int a = kind == PH_ASSEMBLY ? 1 : 0;
  const int tg = kind == PH_ASSEMBLY ? MF_INTERIOR : P.targets;
  const bool acc = kind != PH_SWEEP;
  const int64_t rows = P.rows[a][colour];
  if (rows == 0) return MF_OK;
  const bool timed = allow_timing && ctx->timing && kind != PH_ASSEMBLY;
  if (timed) MF_TRY(timing_begin(ctx, s));
  float* dst = acc ? out : P.u;
  if (P.embed_c) {
    MF_TRY(run_colour_gelu(P, colour, kind, out, s));
  } else if (P.nd == 1) {
    const mf_domain_desc* dom = P.dom;
    PhaseArgs p{P.u + dom->field_offset, dst + dom->field_offset, dom->pitch, dom->units_x,
                dom->units_y, colour};
    const int R = tile_rows_for(ctx, P.width, P.prec, tg, dom, 1, rows);
    MF_HIP(launch_phase(P.net, P.width, P.prec, tg, acc, R, p, s));
  } else {
    MF_HIP(launch_phase_multi(P.net, P.width, P.prec, tg, acc, P.R[a], P.u, dst, P.d_doms,
                              P.d_tb[a] + colour * (P.nd + 1), P.nd, P.n_tiles[a][colour], colour,
                              ctx->n_cu, s));
  }
  if (timed) MF_TRY(timing_end(ctx, s, rows, 1));
  return MF_OK;
}

// One sweep of the plan: the four colour phases in order (multiplicative),
// or the additive form (all placements read u; targets take the mean).
static mf_status run_sweep(mf_ctx* ctx, const Plan& P, hipStream_t s, bool allow_timing = true) {
  if (P.mode == MF_MULTIPLICATIVE) {
    for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, P, c, PH_SWEEP, nullptr, s, allow_timing));
    return MF_OK;
  }
  for (int d = 0; d < P.nd; ++d)
    MF_HIP(launch_additive_init(P.u + P.dom[d].field_offset, P.anext + P.dom[d].field_offset, P.dom[d].pitch,
                                P.dom[d].units_x, P.dom[d].units_y, P.targets, s));
  for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, P, c, PH_ADDITIVE, P.anext, s, allow_timing));
  for (int d = 0; d < P.nd; ++d)
    MF_HIP(launch_additive_copy(P.anext + P.dom[d].field_offset, P.u + P.dom[d].field_offset, P.dom[d].pitch,
                                P.dom[d].units_x, P.dom[d].units_y, P.targets, s));
  return MF_OK;
}

// Cached graph of `sweeps` sweeps on ctx->gstream; captured on first use.
static mf_status sweep_graph(mf_ctx* ctx, const Plan& P, int sweeps, hipGraphExec_t* out) {
  const int64_t pitch = P.nd == 1 ? P.dom->pitch : 0;
  const int ux = P.nd == 1 ? P.dom->units_x : -P.nd;
  const int uy = P.nd == 1 ? P.dom->units_y : (int)(P.key & 0x7fffffff);
  for (const SweepGraph& g : ctx->graphs) {
    if (g.field == P.u && g.ws == P.ws && g.pitch == pitch && g.ux == ux && g.uy == uy &&
        g.key == P.key && g.width == P.width && g.prec == P.prec && g.targets == P.targets &&
        g.mode == P.mode && g.sweeps == sweeps) {
      *out = g.exec;
      return MF_OK;
    }
  }
  if (ctx->graphs.size() >= 16) {   // bounded cache: drop the oldest entry
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  hipGraph_t graph = nullptr;
  MF_HIP(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
  mf_status st = MF_OK;
  for (int k = 0; k < sweeps && st == MF_OK; ++k) st = run_sweep(ctx, P, ctx->gstream, false);
  hipError_t e = hipStreamEndCapture(ctx->gstream, &graph);
  if (st != MF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(MF_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(MF_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
  ctx->graphs.push_back(SweepGraph{P.u, P.ws, pitch, ux, uy, P.width, P.prec, P.targets, P.mode, sweeps,
                                   P.key, exec});
  *out = exec;
  return MF_OK;
}

// max_sweeps sweeps with no delta test, replayed from captured graphs of up
// to kGraphSweeps sweeps on the context's stream, ordered after and before
// the caller's stream by events.
static constexpr int kGraphSweeps = 16;
static mf_status run_sweeps_graph(mf_ctx* ctx, const Plan& P, int max_sweeps, hipStream_t s) {
  const int full = max_sweeps / kGraphSweeps, rem = max_sweeps % kGraphSweeps;
  hipGraphExec_t g_full = nullptr, g_rem = nullptr;
  if (full > 0) MF_TRY(sweep_graph(ctx, P, kGraphSweeps, &g_full));
  if (rem > 0) MF_TRY(sweep_graph(ctx, P, rem, &g_rem));
  int64_t rows_sweep = 0;
  int launches_sweep = 0;
  for (int c = 0; c < 4; ++c) {
    rows_sweep += P.rows[0][c];
    launches_sweep += P.rows[0][c] > 0 ? 1 : 0;
  }
  MF_HIP(hipEventRecord(ctx->fork, s));
  MF_HIP(hipStreamWaitEvent(ctx->gstream, ctx->fork, 0));
  for (int i = 0; i < full + (rem > 0 ? 1 : 0); ++i) {
    const bool last_rem = i == full;
    const int n = last_rem ? rem : kGraphSweeps;
    if (ctx->timing) MF_TRY(timing_begin(ctx, ctx->gstream));
    MF_HIP(hipGraphLaunch(last_rem ? g_rem : g_full, ctx->gstream));
    if (ctx->timing) MF_TRY(timing_end(ctx, ctx->gstream, rows_sweep * n, (int64_t)launches_sweep * n));
  }
  MF_HIP(hipEventRecord(ctx->join, ctx->gstream));
  MF_HIP(hipStreamWaitEvent(s, ctx->join, 0));
  return MF_OK;
}

// Prepared network of either architecture into the layout L.
static hipError_t prepare_net(const mf_sdnet_desc* desc, const float* params, int prec, const NetLayout& L, void* ws,
                              hipStream_t s) {
  if (is_gelu(desc)) return launch_prepare_net_embed(params, desc->width, desc->embed_channels, L, ws, s);
  return launch_prepare_net(params, desc->width, prec, L, ws, s);
}

mf_status mf_sweep(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                   const mf_domain_desc* dom, int32_t n_domains, int32_t colour, int32_t targets,
                   int32_t mode, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  SweepLayout L;
  MF_TRY(sweep_common_checks(desc, params, u, dom, n_domains, targets, mode, prec, ws, ws_bytes, &L));
  if (colour < -1 || colour > 3) return fail(MF_EINVAL, "colour %d not in -1..3", colour);
  if (mode == MF_ADDITIVE && colour != -1)
    return fail(MF_EINVAL, "an additive sweep has no single colour phase (colour must be -1)");
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(prepare_net(desc, params, prec, L.net, ws, s));
  Plan P;
  MF_TRY(make_plan(ctx, desc, prec, targets, mode, u, dom, n_domains, ws, L, s, &P));
  P.params = params;
  if (colour < 0) {
    MF_TRY(run_sweep(ctx, P, s));
  } else {
    MF_TRY(run_colour(ctx, P, colour, PH_SWEEP, nullptr, s));
  }
  return ok();
}

mf_status mf_sweep_noalloc(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                           const mf_domain_desc* dom, int32_t n_domains, int32_t colour, int32_t targets,
                           int32_t prec, void* stream) {
  MF_TRY(check_desc(desc));
  MF_TRY(need_tanh(desc, "mf_sweep_noalloc"));
  MF_TRY(check_prec(prec));
  MF_TRY(check_domain(dom, n_domains));
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(u, "u"));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (colour < -1 || colour > 3) return fail(MF_EINVAL, "colour %d not in -1..3", colour);
  const SweepLayout L = noalloc_layout(desc->width, prec, n_domains);
  if (L.total > kScratchBytes)
    return fail(MF_ENOMEM,
                "%d domains at width %d need %zu bytes of static scratch; the limit is %zu bytes "
                "(use mf_sweep with a workspace)",
                n_domains, desc->width, L.total, kScratchBytes);
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  if (!ctx->scratch) return fail(MF_EDEVICE, "context has no static scratch address");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  void* ws = ctx->scratch;
  MF_HIP(launch_prepare_net(params, desc->width, prec, L.net, ws, s));
  Plan P;
  MF_TRY(make_plan(ctx, desc, prec, targets, MF_MULTIPLICATIVE, u, dom, n_domains, ws, L, s, &P));
  if (colour < 0) {
    MF_TRY(run_sweep(ctx, P, s));
  } else {
    MF_TRY(run_colour(ctx, P, colour, PH_SWEEP, nullptr, s));
  }
  return ok();
}

mf_status mf_autotune(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                      const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t prec,
                      int32_t trials, void* ws, size_t ws_bytes, void* stream, int32_t* rows_out) {
  SweepLayout L;
  MF_TRY(sweep_common_checks(desc, params, u, dom, n_domains, targets, MF_MULTIPLICATIVE, prec, ws,
                             ws_bytes, &L));
  MF_TRY(need_tanh(desc, "mf_autotune (tile shapes of the tanh kernels)"));
  if (trials < 1 || trials > 1000) return fail(MF_EINVAL, "trials %d not in 1..1000", trials);
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_prepare_net(params, desc->width, prec, L.net, ws, s));
  // Candidates. A batch runs the batched kernel, whose streamed-weight fp32
  // form spills (not offered); its 256-row row-split tile comes in both
  // launch forms (one tile per workgroup, or a persistent grid).
  const bool batch = n_domains > 1;
  const int cands_fp32[] = {32, 64, 64 | MF_TILE_STREAM};
  const int cands_bf16[] = {64, 128, 256, 128 | MF_TILE_WIDE, 256 | MF_TILE_WIDE, 256 | MF_TILE_ROWSPLIT,
                            128 | MF_TILE_ROWSPLIT, 256 | MF_TILE_ROWSPLIT | MF_TILE_PERSIST};
  const int cands_fp16[] = {64, 128, 256, 256 | MF_TILE_ROWSPLIT, 128 | MF_TILE_ROWSPLIT,
                            256 | MF_TILE_ROWSPLIT | MF_TILE_PERSIST};
  const int* cands = prec == MF_FP32 ? cands_fp32 : prec == MF_BF16 ? cands_bf16 : cands_fp16;
  const int n_cands = prec == MF_FP32 ? (batch ? 2 : 3) : prec == MF_BF16 ? (batch ? 8 : 7) : (batch ? 6 : 5);
  const int saved_force = ctx->force_rows[prec];
  const bool saved_timing = ctx->timing;
  ctx->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MF_HIP(hipEventCreate(&e0));
  MF_HIP(hipEventCreate(&e1));
  // every candidate: one warm-up sweep; then kTuneRounds rounds that time
  // `trials` sweeps of each candidate in turn, keeping each one's fastest
  // round (interleaving keeps clock ramps and neighbours' noise from
  // favouring whichever shape happens to run first). A batch's plan uploads
  // the tile table of its shape, so it is made again before each timing.
  constexpr int kTuneRounds = 3;
  Plan plan;
  float ms_best[8];
  uint64_t key = 0;
  mf_status st = MF_OK;
  for (int ci = 0; ci < n_cands && st == MF_OK; ++ci) {
    ctx->force_rows[prec] = cands[ci];
    st = make_plan(ctx, desc, prec, targets, MF_MULTIPLICATIVE, u, dom, n_domains, ws, L, s, &plan);
    if (st == MF_OK) st = run_sweep(ctx, plan, s);   // warm-up
    key = plan.key;
    ms_best[ci] = 0.0f;
  }
  for (int round = 0; round < kTuneRounds && st == MF_OK; ++round) {
    for (int ci = 0; ci < n_cands && st == MF_OK; ++ci) {
      ctx->force_rows[prec] = cands[ci];   // the single-domain launch reads the shape from the context
      st = make_plan(ctx, desc, prec, targets, MF_MULTIPLICATIVE, u, dom, n_domains, ws, L, s, &plan);
      if (st != MF_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = fail(MF_EDEVICE, "event record failed"); break; }
      for (int k = 0; k < trials && st == MF_OK; ++k) st = run_sweep(ctx, plan, s);
      if (st != MF_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(MF_EDEVICE, "event timing failed");
        break;
      }
      if (round == 0 || ms < ms_best[ci]) ms_best[ci] = ms;
    }
  }
  int best = 0;
  float best_ms = 0.0f;
  for (int ci = 0; ci < n_cands && st == MF_OK; ++ci)
    if (best == 0 || ms_best[ci] < best_ms) {
      best = cands[ci];
      best_ms = ms_best[ci];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->force_rows[prec] = saved_force;
  ctx->timing = saved_timing;
  if (st != MF_OK) return st;
  const int ux = batch ? 0 : dom->units_x, uy = batch ? 0 : dom->units_y;
  const uint64_t k = batch ? key : 0;
  bool found = false;
  for (TuneEntry& t : ctx->tuned)
    if (t.width == desc->width && t.prec == prec && t.targets == targets && t.ux == ux && t.uy == uy && t.key == k) {
      t.rows = best;
      found = true;
    }
  if (!found) ctx->tuned.push_back(TuneEntry{desc->width, prec, targets, ux, uy, best, k});
  for (SweepGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  if (rows_out) *rows_out = best;
  return ok();
}

// delta over all domains' skeletons: per-domain partial sums, summed on the host.
static mf_status delta_snapshot(const Plan& P, const SweepLayout& L, void* ws, hipStream_t s) {
  char* wsb = static_cast<char*>(ws);
  float* skel = reinterpret_cast<float*>(wsb + L.skel);
  for (int d = 0; d < P.nd; ++d) {
    const mf_domain_desc& D = P.dom[d];
    MF_HIP(launch_skeleton_snapshot(P.u + D.field_offset, D.pitch, D.units_x, D.units_y, skel, s));
    skel += skeleton_count(D.units_x, D.units_y);
  }
  return MF_OK;
}

static mf_status delta_eval(const Plan& P, const SweepLayout& L, void* ws, hipStream_t s, float* num,
                            float* den) {
  char* wsb = static_cast<char*>(ws);
  const float* skel = reinterpret_cast<const float*>(wsb + L.skel);
  float* part = reinterpret_cast<float*>(wsb + L.part);
  float* dres = reinterpret_cast<float*>(wsb + L.dres);
  for (int d = 0; d < P.nd; ++d) {
    const mf_domain_desc& D = P.dom[d];
    MF_HIP(launch_delta(P.u + D.field_offset, D.pitch, D.units_x, D.units_y, skel,
                        part + (size_t)2 * kDeltaBlocks * d, dres + 2 * d, s));
    skel += skeleton_count(D.units_x, D.units_y);
  }
  std::vector<float> h(2 * (size_t)P.nd);
  MF_HIP(hipMemcpyAsync(h.data(), dres, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  double sn = 0.0, sd = 0.0;
  for (int d = 0; d < P.nd; ++d) {
    sn += h[2 * d];
    sd += h[2 * d + 1];
  }
  *num = (float)sn;
  *den = (float)sd;
  return MF_OK;
}

mf_status mf_solve(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                   const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t mode,
                   int32_t prec, int32_t max_sweeps, float eps, int32_t check_every, int32_t flags,
                   float* u_out, int32_t* sweeps_done, float* last_delta, void* ws, size_t ws_bytes,
                   void* stream) {
  SweepLayout L;
  MF_TRY(sweep_common_checks(desc, params, u, dom, n_domains, targets, mode, prec, ws, ws_bytes, &L));
  if (max_sweeps < 0) return fail(MF_EINVAL, "max_sweeps %d < 0", max_sweeps);
  if (!(eps >= 0.0f) || isinf(eps)) return fail(MF_EINVAL, "eps must be finite and >= 0");
  if (eps > 0.0f && check_every < 1) return fail(MF_EINVAL, "check_every %d < 1", check_every);
  if (flags & ~MF_SOLVE_FAIL_IF_NOT_CONVERGED) return fail(MF_EINVAL, "unknown flags 0x%x", flags);
  if (u_out) {
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
  }
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(prepare_net(desc, params, prec, L.net, ws, s));
  Plan P;
  MF_TRY(make_plan(ctx, desc, prec, targets, mode, u, dom, n_domains, ws, L, s, &P));
  P.params = params;

  int done = 0;
  float last = NAN;
  bool converged = false;
  const bool inject = ctx->fault_sweep > 0 && mode == MF_MULTIPLICATIVE;
  if (eps == 0.0f && ctx->use_graphs && max_sweeps > 0 && !inject && !P.embed_c) {
    MF_TRY(run_sweeps_graph(ctx, P, max_sweeps, s));
    done = max_sweeps;
  }
  for (int k = done + 1; k <= max_sweeps; ++k) {
    const bool check = eps > 0.0f && (k % check_every) == 0;
    if (check) MF_TRY(delta_snapshot(P, L, ws, s));
    if (inject && k == ctx->fault_sweep) {
      for (int c = 0; c < ctx->fault_colour; ++c) MF_TRY(run_colour(ctx, P, c, PH_SWEEP, nullptr, s));
      return fail(MF_EDEVICE, "injected fault (MF_FAULT_INJECT) before colour %d of sweep %d", ctx->fault_colour,
                  k);
    }
    MF_TRY(run_sweep(ctx, P, s));
    done = k;
    if (check) {
      float num = 0.0f, den = 0.0f;
      MF_TRY(delta_eval(P, L, ws, s, &num, &den));
      if (den == 0.0f) {
        last = INFINITY;
      } else {
        last = sqrtf(num) / sqrtf(den);
        if (!isfinite(last)) return fail(MF_ENONFINITE, "delta is not finite after sweep %d", k);
      }
      if (last < eps) {
        converged = true;
        break;
      }
    }
  }
  if (u_out) {
    for (int d = 0; d < n_domains; ++d)
      MF_HIP(launch_assembly_init(u + dom[d].field_offset, u_out + dom[d].field_offset, dom[d].pitch,
                                  dom[d].units_x, dom[d].units_y, s));
    for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, P, c, PH_ASSEMBLY, u_out, s));
  }
  if (sweeps_done || last_delta) MF_HIP(hipStreamSynchronize(s));
  if (sweeps_done) *sweeps_done = done;
  if (last_delta) *last_delta = last;
  if ((flags & MF_SOLVE_FAIL_IF_NOT_CONVERGED) && eps > 0.0f && !converged)
    return fail(MF_ENOTCONVERGED, "delta %g still >= eps %g after %d sweeps", (double)last, (double)eps, done);
  return ok();
}

// ---------------------------------------------------------------------------
// mf_solve_mixed: 16-bit sweeps with a float32 correction refreshed every
// `refresh_every` sweeps (the refresh sweep itself runs in float32).
// ---------------------------------------------------------------------------
struct MixLayout {
  SweepLayout l16, l16t, l32;          // each relative to its own sub-workspace
  size_t o16 = 0, o16t = 0, o32 = 0;   // sub-workspace offsets
  size_t tmp = 0, corr = 0, table = 0, total = 0;
  int64_t lo = 0;
  size_t span = 0;                     // floats per field copy (hi - lo)
};

static MixLayout mixed_layout(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int nd, int prec,
                              std::vector<mf_domain_desc>* dint) {
  MixLayout M;
  int64_t lo = INT64_MAX, hi = 0;
  for (int i = 0; i < nd; ++i) {
    lo = std::min<int64_t>(lo, dom[i].field_offset);
    hi = std::max<int64_t>(hi, dom[i].field_offset + field_extent(dom[i]));
  }
  M.lo = lo;
  M.span = (size_t)(hi - lo);
  std::vector<mf_domain_desc> di(dom, dom + nd);
  for (mf_domain_desc& e : di) e.field_offset -= lo;
  M.l16 = sweep_layout(desc->width, prec, dom, nd, MF_MULTIPLICATIVE);
  M.l16t = sweep_layout(desc->width, prec, di.data(), nd, MF_MULTIPLICATIVE);
  M.l32 = sweep_layout(desc->width, MF_FP32, dom, nd, MF_MULTIPLICATIVE);
  size_t o = 0;
  M.o16 = o; o = align256(o + M.l16.total);
  M.o16t = o; o = align256(o + M.l16t.total);
  M.o32 = o; o = align256(o + M.l32.total);
  M.tmp = o; o = align256(o + M.span * 4);
  M.corr = o; o = align256(o + 4 * M.span * 4);
  M.table = o; o = align256(o + (size_t)nd * sizeof(DomEntry) + 4 * ((size_t)nd + 1) * 4);
  M.total = o;
  if (dint) *dint = di;
  return M;
}

static mf_status mixed_checks(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int nd, int targets, int prec) {
  MF_TRY(check_desc(desc));
  MF_TRY(need_tanh(desc, "mf_solve_mixed"));
  MF_TRY(check_domain(dom, nd));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (prec != MF_BF16 && prec != MF_FP16) return fail(MF_EINVAL, "mf_solve_mixed: prec must be MF_BF16 or MF_FP16");
  int64_t n_place = 0;
  for (int d = 0; d < nd; ++d) n_place += (int64_t)dom[d].units_x * dom[d].units_y;
  if (n_place > INT32_MAX) return fail(MF_ESHAPE, "batch has too many placements");
  return MF_OK;
}

mf_status mf_mixed_ws_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                           int32_t targets, int32_t prec, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(mixed_checks(desc, dom, n_domains, targets, prec));
  *bytes = mixed_layout(desc, dom, n_domains, prec, nullptr).total;
  return ok();
}

mf_status mf_solve_mixed(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, float* u,
                         const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t prec,
                         int32_t max_sweeps, int32_t refresh_every, int32_t assembly_prec, float* u_out, void* ws,
                         size_t ws_bytes, void* stream) {
  MF_TRY(mixed_checks(desc, dom, n_domains, targets, prec));
  if (assembly_prec != MF_FP32 && assembly_prec != prec)
    return fail(MF_EINVAL, "assembly_prec must be MF_FP32 or the sweeps' precision");
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(u, "u"));
  if (max_sweeps < 0) return fail(MF_EINVAL, "max_sweeps %d < 0", max_sweeps);
  if (refresh_every < 1) return fail(MF_EINVAL, "refresh_every %d < 1", refresh_every);
  if (u_out) {
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
  }
  std::vector<mf_domain_desc> dint;
  const MixLayout M = mixed_layout(desc, dom, n_domains, prec, &dint);
  MF_TRY(check_ws(ws, ws_bytes, M.total));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  char* b = static_cast<char*>(ws);
  void* w16 = b + M.o16;
  void* w16t = b + M.o16t;
  void* w32 = b + M.o32;
  float* tmp = reinterpret_cast<float*>(b + M.tmp);
  float* corr = reinterpret_cast<float*>(b + M.corr);
  const int nd = n_domains;
  MF_HIP(prepare_net(desc, params, prec, M.l16.net, w16, s));
  MF_HIP(prepare_net(desc, params, prec, M.l16t.net, w16t, s));
  MF_HIP(prepare_net(desc, params, MF_FP32, M.l32.net, w32, s));
  Plan P16, P16t, P32;
  MF_TRY(make_plan(ctx, desc, prec, targets, MF_MULTIPLICATIVE, u, dom, nd, w16, M.l16, s, &P16));
  MF_TRY(make_plan(ctx, desc, prec, targets, MF_MULTIPLICATIVE, tmp, dint.data(), nd, w16t, M.l16t, s, &P16t));
  MF_TRY(make_plan(ctx, desc, MF_FP32, targets, MF_MULTIPLICATIVE, u, dom, nd, w32, M.l32, s, &P32));
  // the correction kernels' table: the caller's offsets and per-colour
  // placement prefixes
  std::vector<char> host((size_t)nd * sizeof(DomEntry) + 4 * ((size_t)nd + 1) * 4);
  DomEntry* he = reinterpret_cast<DomEntry*>(host.data());
  int32_t* hq = reinterpret_cast<int32_t*>(host.data() + (size_t)nd * sizeof(DomEntry));
  int64_t n_place[4] = {0, 0, 0, 0};
  for (int d = 0; d < nd; ++d) he[d] = DomEntry{dom[d].field_offset, dom[d].pitch, dom[d].units_x, dom[d].units_y};
  for (int c = 0; c < 4; ++c) {
    int32_t acc = 0;
    for (int d = 0; d < nd; ++d) {
      hq[c * (nd + 1) + d] = acc;
      acc += (dom[d].units_x - (c & 1)) * (dom[d].units_y - (c >> 1));
    }
    hq[c * (nd + 1) + nd] = acc;
    n_place[c] = acc;
  }
  char* tb = b + M.table;
  MF_HIP(hipMemcpyAsync(tb, host.data(), host.size(), hipMemcpyHostToDevice, s));
  const DomEntry* d_doms = reinterpret_cast<const DomEntry*>(tb);
  const int32_t* d_q = reinterpret_cast<const int32_t*>(tb + (size_t)nd * sizeof(DomEntry));

  for (int k = 0; k < max_sweeps; ++k) {
    const bool refresh = k % refresh_every == 0;
    for (int c = 0; c < 4; ++c) {
      if (n_place[c] == 0) continue;
      const int32_t* qc = d_q + c * (nd + 1);
      float* cc = corr + (size_t)c * M.span;
      if (refresh) {
        // the same field state in both precisions: the 16-bit phase runs on a copy
        MF_HIP(hipMemcpyAsync(tmp, u + M.lo, M.span * 4, hipMemcpyDeviceToDevice, s));
        MF_TRY(run_colour(ctx, P32, c, PH_SWEEP, nullptr, s));
        MF_TRY(run_colour(ctx, P16t, c, PH_SWEEP, nullptr, s, false));
        MF_HIP(launch_corr_targets(targets, 0, u, tmp, cc, M.lo, d_doms, qc, nd, c, n_place[c], s));
      } else {
        MF_TRY(run_colour(ctx, P16, c, PH_SWEEP, nullptr, s));
        MF_HIP(launch_corr_targets(targets, 1, u, tmp, cc, M.lo, d_doms, qc, nd, c, n_place[c], s));
      }
    }
  }
  if (u_out) {   // the assembly in float32 or in the sweeps' precision
    const Plan& PA = assembly_prec == MF_FP32 ? P32 : P16;
    for (int d = 0; d < nd; ++d)
      MF_HIP(launch_assembly_init(u + dom[d].field_offset, u_out + dom[d].field_offset, dom[d].pitch,
                                  dom[d].units_x, dom[d].units_y, s));
    for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, PA, c, PH_ASSEMBLY, u_out, s));
  }
  return ok();
}

mf_status mf_sweep_operator(mf_ctx* ctx, const float* Hop, int64_t hop_rows, int32_t targets,
                            float* u, float* u_out, const mf_domain_desc* dom, int32_t colour,
                            void* stream) {
  MF_TRY(check_ptr(Hop, "Hop"));
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_domain(dom, 1));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (colour < -1 || colour > 4) return fail(MF_EINVAL, "colour %d not in -1..4", colour);
  if (hop_rows != (targets == MF_CROSS ? 61 : 961))
    return fail(MF_ESHAPE, "Hop has %lld rows; the target set needs %d", (long long)hop_rows,
                targets == MF_CROSS ? 61 : 961);
  if (colour == 4) {
    if (targets != MF_INTERIOR) return fail(MF_EINVAL, "assembly needs the INTERIOR operator");
    MF_TRY(check_ptr(u_out, "u_out"));
    if (u_out == u) return fail(MF_EINVAL, "u_out must not alias u");
  }
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  float* field = u + dom->field_offset;
  if (colour == 4) {
    float* out = u_out + dom->field_offset;
    MF_HIP(launch_assembly_init(field, out, dom->pitch, dom->units_x, dom->units_y, s));
    for (int c = 0; c < 4; ++c) {
      PhaseArgs p{field, out, dom->pitch, dom->units_x, dom->units_y, c};
      MF_HIP(launch_operator_phase(Hop, MF_INTERIOR, true, p, s));
    }
    return ok();
  }
  for (int c = (colour < 0 ? 0 : colour); c <= (colour < 0 ? 3 : colour); ++c) {
    PhaseArgs p{field, field, dom->pitch, dom->units_x, dom->units_y, c};
    MF_HIP(launch_operator_phase(Hop, targets, false, p, s));
  }
  return ok();
}

// ---------------------------------------------------------------------------
// One colour's gather and scatter as standalone calls
// ---------------------------------------------------------------------------
int64_t mf_colour_placements(const mf_domain_desc* dom, int32_t colour) {
  if (!dom || colour < 0 || colour > 3 || check_one_domain(dom, 0) != MF_OK) return -1;
  return (int64_t)(dom->units_x - (colour & 1)) * (dom->units_y - (colour >> 1));
}

mf_status mf_target_coords(int32_t targets, float* X_host) {
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (!X_host) return fail(MF_EINVAL, "X_host is NULL");
  if (targets == MF_CROSS) {
    int t = 0;
    for (int j = 1; j <= 31; ++j, ++t) { X_host[2 * t] = 0.5f; X_host[2 * t + 1] = j / 32.0f; }
    for (int i = 1; i <= 31; ++i) {
      if (i == 16) continue;
      X_host[2 * t] = i / 32.0f;
      X_host[2 * t + 1] = 0.5f;
      ++t;
    }
  } else {
    for (int j = 1, t = 0; j <= 31; ++j)
      for (int i = 1; i <= 31; ++i, ++t) { X_host[2 * t] = i / 32.0f; X_host[2 * t + 1] = j / 32.0f; }
  }
  return ok();
}

static mf_status check_colour_io(const mf_domain_desc* dom, int32_t colour) {
  MF_TRY(check_domain(dom, 1));
  if (colour < 0 || colour > 3) return fail(MF_EINVAL, "colour %d not in 0..3", colour);
  return MF_OK;
}

mf_status mf_gather(mf_ctx* ctx, const float* u, const mf_domain_desc* dom, int32_t colour, float* G,
                    void* stream) {
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_colour_io(dom, colour));
  const int64_t n_q = mf_colour_placements(dom, colour);
  if (n_q == 0) return ok();   // a one-unit-wide domain has no placements of some colours
  MF_TRY(check_ptr(G, "G"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_gather_colour(u + dom->field_offset, dom->pitch, dom->units_x, colour, n_q, G,
                              static_cast<hipStream_t>(stream)));
  return ok();
}

mf_status mf_scatter(mf_ctx* ctx, const float* pred, int32_t targets, float* u, const mf_domain_desc* dom,
                     int32_t colour, void* stream) {
  MF_TRY(check_ptr(u, "u"));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  MF_TRY(check_colour_io(dom, colour));
  const int64_t n_q = mf_colour_placements(dom, colour);
  if (n_q == 0) return ok();
  MF_TRY(check_ptr(pred, "pred"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_scatter_colour(pred, targets, u + dom->field_offset, dom->pitch, dom->units_x, colour, n_q,
                               static_cast<hipStream_t>(stream)));
  return ok();
}

int64_t mf_skeleton_cols_size(const mf_domain_desc* dom) {
  if (check_domain(dom, 1) != MF_OK) return -1;
  return (int64_t)(2 * dom->units_x + 1) * skel_cols_pitch(dom->units_y);
}

mf_status mf_skeleton_pack(mf_ctx* ctx, const float* u, const mf_domain_desc* dom, float* cols, void* stream) {
  MF_TRY(check_domain(dom, 1));
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_ptr(cols, "cols"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_skel_pack(u + dom->field_offset, dom->pitch, dom->units_x, dom->units_y, cols,
                          static_cast<hipStream_t>(stream)));
  return ok();
}

mf_status mf_skeleton_unpack(mf_ctx* ctx, const float* cols, float* u, const mf_domain_desc* dom, void* stream) {
  MF_TRY(check_domain(dom, 1));
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_ptr(cols, "cols"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_skel_unpack(cols, u + dom->field_offset, dom->pitch, dom->units_x, dom->units_y,
                            static_cast<hipStream_t>(stream)));
  return ok();
}

mf_status mf_gather_skel(mf_ctx* ctx, const float* u, const float* cols, const mf_domain_desc* dom, int32_t colour,
                         float* G, void* stream) {
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_colour_io(dom, colour));
  MF_TRY(check_ptr(cols, "cols"));
  const int64_t n_q = mf_colour_placements(dom, colour);
  if (n_q == 0) return ok();
  MF_TRY(check_ptr(G, "G"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_gather_skel(u + dom->field_offset, dom->pitch, cols, dom->units_x, dom->units_y, colour, n_q, G,
                            static_cast<hipStream_t>(stream)));
  return ok();
}

mf_status mf_scatter_skel(mf_ctx* ctx, const float* pred, float* u, float* cols, const mf_domain_desc* dom,
                          int32_t colour, void* stream) {
  MF_TRY(check_ptr(u, "u"));
  MF_TRY(check_colour_io(dom, colour));
  MF_TRY(check_ptr(cols, "cols"));
  const int64_t n_q = mf_colour_placements(dom, colour);
  if (n_q == 0) return ok();
  MF_TRY(check_ptr(pred, "pred"));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_scatter_skel(pred, u + dom->field_offset, dom->pitch, cols, dom->units_x, dom->units_y, colour, n_q,
                             static_cast<hipStream_t>(stream)));
  return ok();
}

// ---------------------------------------------------------------------------
// mf_solve_adjoint
// ---------------------------------------------------------------------------
static constexpr int64_t kAdjRows = 262144;   // (placement, target) rows per chunk

// Workspace of mf_solve_adjoint. The field copies (the running field, the
// checkpoints, the per-phase states of one segment and the assembly) cover the
// span [lo, hi) that the domains occupy in the caller's buffer, each domain at
// its own offset minus lo, so that one copy moves every domain of the batch.
struct AdjLayout {
  NetLayout net;
  size_t whT = 0, X_cross = 0, X_interior = 0, G = 0, C = 0, ubp = 0, Z[4] = {0, 0, 0, 0}, Ab[2] = {0, 0}, Sv[4] = {0, 0, 0, 0};
  size_t csum = 0, gb = 0, part = 0, ftable = 0, atable = 0, field = 0, ckpt = 0, states = 0, uout = 0, total = 0;
  size_t gC = 0, gX = 0, gZ[2] = {0, 0};   // the GELU network's forward phases (as in the sweep workspace)
  int64_t lo = 0;       // first float of the span
  size_t fsize = 0;     // floats per field copy (hi - lo)
  int n_ckpt = 0;
};

static AdjLayout adjoint_layout(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int nd, int K,
                                int ckpt_every) {
  AdjLayout A;
  const int width = desc->width;
  const bool gelu = is_gelu(desc);
  A.net = net_layout(width, MF_FP32, 0, gelu ? 128 * desc->embed_channels : 128);
  const size_t d = (size_t)width;
  const size_t max_q = (size_t)(kAdjRows / 61);
  int64_t lo = INT64_MAX, hi = 0;
  for (int i = 0; i < nd; ++i) {
    lo = std::min<int64_t>(lo, dom[i].field_offset);
    hi = std::max<int64_t>(hi, dom[i].field_offset + field_extent(dom[i]));
  }
  A.lo = lo;
  A.fsize = (size_t)(hi - lo);
  A.n_ckpt = K > 0 ? (K + ckpt_every - 1) / ckpt_every : 0;
  size_t o = A.net.end;
  A.whT = o; o = align256(o + 3 * d * d * 4);
  A.X_cross = o; o = align256(o + 61 * 2 * 4);
  A.X_interior = o; o = align256(o + 961 * 2 * 4);
  A.G = o; o = align256(o + max_q * 128 * 4);
  A.C = o; o = align256(o + max_q * d * 4);
  A.ubp = o; o = align256(o + (size_t)kAdjRows * 4);
  for (int l = 0; l < 4; ++l) { A.Z[l] = o; o = align256(o + (size_t)kAdjRows * d * 4); }
  for (int l = 0; l < 2; ++l) { A.Ab[l] = o; o = align256(o + (size_t)kAdjRows * d * 4); }
  if (gelu)   // the GELU network's saved pre-activations
    for (int l = 0; l < 4; ++l) { A.Sv[l] = o; o = align256(o + (size_t)kAdjRows * d * 4); }
  A.csum = o; o = align256(o + 3 * max_q * d * 4);
  A.gb = o; o = align256(o + max_q * 128 * 4);
  A.part = o; o = align256(o + 1024 * 4);
  // the forward plan's batch table (as in the sweep workspace) and the
  // adjoint's: DomEntry [nd] + placement prefixes [4][nd + 1]
  A.ftable = o; o = align256(o + (size_t)nd * sizeof(DomEntry) + 2 * 4 * ((size_t)nd + 1) * 4);
  A.atable = o; o = align256(o + (size_t)nd * sizeof(DomEntry) + 4 * ((size_t)nd + 1) * 4);
  if (gelu) {   // the forward solve's GELU phase chunks, sized as in sweep_layout
    A.gC = o; o = align256(o + (size_t)(kGeluRows / 61) * width * 4);
    A.gX = o; o = align256(o + (61 + 961) * 2 * 4);
    for (int l = 0; l < 2; ++l) { A.gZ[l] = o; o = align256(o + (size_t)kGeluRows * width * 4); }
  }
  A.field = o; o = align256(o + A.fsize * 4);
  A.ckpt = o; o = align256(o + (size_t)A.n_ckpt * A.fsize * 4);
  A.states = o; o = align256(o + 4 * (size_t)ckpt_every * A.fsize * 4);
  A.uout = o; o = align256(o + A.fsize * 4);
  A.total = o;
  return A;
}

static mf_status adjoint_checks(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int nd, int targets,
                                int K, int ckpt_every) {
  MF_TRY(check_desc(desc));
  MF_TRY(check_domain(dom, nd));
  if (targets != MF_CROSS && targets != MF_INTERIOR) return fail(MF_EINVAL, "targets %d unknown", targets);
  if (K < 0) return fail(MF_EINVAL, "K %d < 0", K);
  if (ckpt_every < 1 || ckpt_every > 1000) return fail(MF_EINVAL, "ckpt_every %d not in 1..1000", ckpt_every);
  int64_t n_place = 0;
  for (int d = 0; d < nd; ++d) n_place += (int64_t)dom[d].units_x * dom[d].units_y;
  if (n_place > INT32_MAX) return fail(MF_ESHAPE, "batch has too many placements");
  return MF_OK;
}

mf_status mf_adjoint_ws_size(const mf_sdnet_desc* desc, const mf_domain_desc* dom, int32_t n_domains,
                             int32_t targets, int32_t K, int32_t ckpt_every, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(adjoint_checks(desc, dom, n_domains, targets, K, ckpt_every));
  *bytes = adjoint_layout(desc, dom, n_domains, K, ckpt_every).total;
  return ok();
}

// The K sweeps and the assembly run forward with checkpoints on a copy of the
// domains' span, batched as mf_solve batches them; the reverse then takes
// every domain's placements of a colour in the same launches.
mf_status mf_solve_adjoint(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* u0,
                           const mf_domain_desc* dom, int32_t n_domains, int32_t targets, int32_t K,
                           int32_t ckpt_every, const float* uout_bar, float* u_out, float* J, float* u0_bar,
                           void* ws, size_t ws_bytes, void* stream) {
  MF_TRY(adjoint_checks(desc, dom, n_domains, targets, K, ckpt_every));
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(u0, "u0"));
  MF_TRY(check_ptr(u0_bar, "u0_bar"));
  if (u_out) MF_TRY(check_ptr(u_out, "u_out"));
  if (J) MF_TRY(check_ptr(J, "J"));
  if (uout_bar) MF_TRY(check_ptr(uout_bar, "uout_bar"));
  if (u0_bar == u0 || (u_out && (u_out == u0 || u_out == u0_bar)))
    return fail(MF_EINVAL, "u0, u_out and u0_bar must be distinct buffers");
  if (uout_bar && (uout_bar == u0_bar || uout_bar == u_out))
    return fail(MF_EINVAL, "uout_bar must not alias u0_bar or u_out");
  const AdjLayout A = adjoint_layout(desc, dom, n_domains, K, ckpt_every);
  MF_TRY(check_ws(ws, ws_bytes, A.total));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  char* b = static_cast<char*>(ws);
  const int nd = n_domains;
  MF_HIP(prepare_net(desc, params, MF_FP32, A.net, ws, s));
  const NetPtrs net = net_ptrs(A.net, ws);
  float* whT = reinterpret_cast<float*>(b + A.whT);
  const bool gelu = is_gelu(desc);
  const int64_t n_in = gelu ? 128 * (int64_t)desc->embed_channels : desc->n_boundary;
  const int64_t off_w2 = (gelu ? embed_param_offset(desc->embed_channels) : 0) + desc->width * (n_in + 2) + desc->width;
  MF_HIP(launch_prepare_wT(params, off_w2, desc->width, whT, s));
  AdjointBuffers ab;
  if (gelu) {
    ab.params = params;
    ab.channels = desc->embed_channels;
    for (int l = 0; l < 4; ++l) ab.Sv[l] = reinterpret_cast<float*>(b + A.Sv[l]);
  }
  ab.X_cross = reinterpret_cast<float*>(b + A.X_cross);
  ab.X_interior = reinterpret_cast<float*>(b + A.X_interior);
  ab.G = reinterpret_cast<float*>(b + A.G);
  ab.C = reinterpret_cast<float*>(b + A.C);
  ab.ubp = reinterpret_cast<float*>(b + A.ubp);
  for (int l = 0; l < 4; ++l) ab.Z[l] = reinterpret_cast<float*>(b + A.Z[l]);
  for (int l = 0; l < 2; ++l) ab.Ab[l] = reinterpret_cast<float*>(b + A.Ab[l]);
  ab.csum = reinterpret_cast<float*>(b + A.csum);
  ab.gb = reinterpret_cast<float*>(b + A.gb);
  ab.max_rows = kAdjRows;
  MF_HIP(launch_target_coords(ab.X_cross, ab.X_interior, s));
  float* part = reinterpret_cast<float*>(b + A.part);
  float* F = reinterpret_cast<float*>(b + A.field);
  float* ckpt = reinterpret_cast<float*>(b + A.ckpt);
  float* states = reinterpret_cast<float*>(b + A.states);
  float* uo = reinterpret_cast<float*>(b + A.uout);
  const size_t fbytes = A.fsize * 4;
  const int64_t lo = A.lo;

  // forward plan on the span copy (domain offsets relative to lo)
  std::vector<mf_domain_desc> dint(dom, dom + nd);
  for (mf_domain_desc& e : dint) e.field_offset -= lo;
  SweepLayout SL;
  SL.net = A.net;
  SL.table = A.ftable;
  SL.gC = A.gC;
  SL.gX = A.gX;
  SL.gZ[0] = A.gZ[0];
  SL.gZ[1] = A.gZ[1];
  Plan P;
  MF_TRY(make_plan(ctx, desc, MF_FP32, targets, MF_MULTIPLICATIVE, F, dint.data(), nd, ws, SL, s, &P));
  P.params = params;   // the GELU network's phases read its convolutions from here
  // the adjoint's table: caller offsets and per-colour placement prefixes
  std::vector<char> host((size_t)nd * sizeof(DomEntry) + 4 * ((size_t)nd + 1) * 4);
  DomEntry* he = reinterpret_cast<DomEntry*>(host.data());
  int32_t* hq = reinterpret_cast<int32_t*>(host.data() + (size_t)nd * sizeof(DomEntry));
  int n_place[4] = {0, 0, 0, 0};
  for (int d = 0; d < nd; ++d) he[d] = DomEntry{dom[d].field_offset, dom[d].pitch, dom[d].units_x, dom[d].units_y};
  for (int c = 0; c < 4; ++c) {
    int32_t acc = 0;
    for (int d = 0; d < nd; ++d) {
      hq[c * (nd + 1) + d] = acc;
      acc += (dom[d].units_x - (c & 1)) * (dom[d].units_y - (c >> 1));
    }
    hq[c * (nd + 1) + nd] = acc;
    n_place[c] = acc;
  }
  char* at = b + A.atable;
  MF_HIP(hipMemcpyAsync(at, host.data(), host.size(), hipMemcpyHostToDevice, s));
  const DomEntry* d_doms = reinterpret_cast<const DomEntry*>(at);
  const int32_t* d_q = reinterpret_cast<const int32_t*>(at + (size_t)nd * sizeof(DomEntry));

  // forward with checkpoints
  MF_HIP(hipMemcpyAsync(F, u0 + lo, fbytes, hipMemcpyDeviceToDevice, s));
  for (int i = 0; i < A.n_ckpt; ++i) {
    MF_HIP(hipMemcpyAsync(ckpt + (size_t)i * A.fsize, F, fbytes, hipMemcpyDeviceToDevice, s));
    const int n_s = std::min(ckpt_every, K - i * ckpt_every);
    for (int k = 0; k < n_s; ++k)
      for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, P, c, PH_SWEEP, nullptr, s, false));
  }
  for (int d = 0; d < nd; ++d) {
    const mf_domain_desc& D = dint[d];
    MF_HIP(launch_assembly_init(F + D.field_offset, uo + D.field_offset, D.pitch, D.units_x, D.units_y, s));
  }
  for (int c = 0; c < 4; ++c) MF_TRY(run_colour(ctx, P, c, PH_ASSEMBLY, uo, s, false));
  for (int d = 0; d < nd; ++d) {
    const mf_domain_desc& D = dom[d];
    const float* uod = uo + dint[d].field_offset;
    const float* seed = uout_bar ? uout_bar + D.field_offset : nullptr;
    if (u_out)
      MF_HIP(hipMemcpy2DAsync(u_out + D.field_offset, D.pitch * 4, uod, D.pitch * 4, (32 * (size_t)D.units_x + 1) * 4,
                              32 * (size_t)D.units_y + 1, hipMemcpyDeviceToDevice, s));
    if (J && seed)
      MF_HIP(launch_grid_dot(seed, uod, D.pitch, D.units_x, D.units_y, part, J, d > 0 ? 1 : 0, s));
    else if (J)
      MF_HIP(launch_interior_sumsq(uod, D.pitch, D.units_x, D.units_y, part, J, d > 0 ? 1 : 0, s));
    // the ring of u_out is u0's, so a seed's ring passes straight to u0_bar
    float* ub = u0_bar + D.field_offset;
    if (seed)
      MF_HIP(launch_assembly_init(seed, ub, D.pitch, D.units_x, D.units_y, s));
    else
      MF_HIP(launch_fill2d(ub, D.pitch, D.units_x, D.units_y, 0.0f, s));
  }
  // reverse: the assembly, then the sweeps segment by segment
  const int w = desc->width;
  for (int c = 3; c >= 0; --c)
    MF_HIP(launch_adjoint_colour(net, w, whT, ab, F, lo, uout_bar ? uout_bar : uo, uout_bar ? 0 : lo, u0_bar,
                                 d_doms, d_q, nd, n_place[c], c, targets, uout_bar ? ADJ_SEED : ADJ_SUMSQ, s));
  for (int i = A.n_ckpt - 1; i >= 0; --i) {
    const int n_s = std::min(ckpt_every, K - i * ckpt_every);
    MF_HIP(hipMemcpyAsync(F, ckpt + (size_t)i * A.fsize, fbytes, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < n_s; ++k)
      for (int c = 0; c < 4; ++c) {
        MF_HIP(hipMemcpyAsync(states + (size_t)(4 * k + c) * A.fsize, F, fbytes, hipMemcpyDeviceToDevice, s));
        MF_TRY(run_colour(ctx, P, c, PH_SWEEP, nullptr, s, false));
      }
    for (int k = n_s - 1; k >= 0; --k)
      for (int c = 3; c >= 0; --c)
        MF_HIP(launch_adjoint_colour(net, w, whT, ab, states + (size_t)(4 * k + c) * A.fsize, lo, nullptr, 0,
                                     u0_bar, d_doms, d_q, nd, n_place[c], c, targets, ADJ_SWEEP, s));
  }
  return ok();
}

// ---------------------------------------------------------------------------
// sdnet_forward
// ---------------------------------------------------------------------------
// Workspace of sdnet_forward: prepared network, projections C [n_bc][d] and,
// for derivative outputs, two stream-row buffers [4 n_bc n_pts][d].
// The GELU network always runs the row kernels: two value-row buffers
// [n_bc n_pts][d] without derivatives.
static size_t forward_ws(int width, int prec, int64_t n_bc, int64_t n_pts, bool derivs, int embed_c,
                         NetLayout* Lout, size_t* c_off, size_t* z_off) {
  NetLayout L = net_layout(width, prec, 0, embed_c ? embed_c * 128 : 128);
  size_t o = L.end;
  *c_off = o;
  o = align256(o + (size_t)n_bc * width * 4);
  *z_off = o;
  if (derivs) o = align256(o + 2 * (size_t)4 * n_bc * n_pts * width * 4);
  else if (embed_c) o = align256(o + 2 * (size_t)n_bc * n_pts * width * 4);
  if (Lout) *Lout = L;
  return o;
}

mf_status sdnet_forward_ws_size(const mf_sdnet_desc* desc, int64_t n_bc, int64_t n_pts,
                                int32_t derivatives, int32_t prec, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  if (n_bc < 0 || n_pts < 0) return fail(MF_ESHAPE, "n_bc and n_pts must be >= 0");
  MF_TRY(gelu_limits(desc, prec, MF_MULTIPLICATIVE));
  size_t c_off, z_off;
  *bytes = forward_ws(desc->width, prec, n_bc, n_pts, derivatives != 0, desc->embed_channels, nullptr, &c_off,
                      &z_off);
  return ok();
}

mf_status sdnet_forward(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* G,
                        int64_t n_bc, const float* X, int64_t n_pts, int32_t x_per_bc, float* U,
                        float* dU, float* lapU, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  MF_TRY(check_desc(desc));
  MF_TRY(check_prec(prec));
  if (n_bc < 0 || n_pts < 0) return fail(MF_ESHAPE, "n_bc and n_pts must be >= 0");
  if (x_per_bc != 0 && x_per_bc != 1) return fail(MF_EINVAL, "x_per_bc must be 0 or 1");
  if (n_bc * n_pts > (1LL << 40)) return fail(MF_ESHAPE, "too many rows");
  const bool derivs = dU || lapU;
  if (derivs && prec != MF_FP32) return fail(MF_EUNSUPPORTED, "derivative outputs need MF_FP32");
  MF_TRY(gelu_limits(desc, prec, MF_MULTIPLICATIVE));
  if (n_bc == 0 || n_pts == 0) return ctx ? ok() : fail(MF_EINVAL, "ctx is NULL");
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(G, "G"));
  MF_TRY(check_ptr(X, "X"));
  MF_TRY(check_ptr(U, "U"));
  if (dU) MF_TRY(check_ptr(dU, "dU"));
  if (lapU) MF_TRY(check_ptr(lapU, "lapU"));
  NetLayout L;
  size_t c_off, z_off;
  const size_t need = forward_ws(desc->width, prec, n_bc, n_pts, derivs, desc->embed_channels, &L, &c_off, &z_off);
  MF_TRY(check_ws(ws, ws_bytes, need));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(prepare_net(desc, params, prec, L, ws, s));
  const NetPtrs net = net_ptrs(L, ws);
  float* C = reinterpret_cast<float*>(static_cast<char*>(ws) + c_off);
  const bool gelu = is_gelu(desc);
  if (gelu)
    MF_HIP(launch_embed_project(params, desc->width, desc->embed_channels, net, G, n_bc, nullptr, 0, 0, 0, 0, C, s));
  else
    MF_HIP(launch_projection(net, desc->width, G, n_bc, C, s));
  float* Z0 = reinterpret_cast<float*>(static_cast<char*>(ws) + z_off);
  if (derivs) {
    float* Z1 = Z0 + (size_t)4 * n_bc * n_pts * desc->width;
    MF_HIP(launch_forward_derivs(net, desc->width, gelu ? ACT_GELU : ACT_TANH, C, X, x_per_bc, n_bc, n_pts, Z0, Z1,
                                 U, dU, lapU, s));
  } else if (gelu) {
    float* Z1 = Z0 + (size_t)n_bc * n_pts * desc->width;
    float* Z[4] = {Z0, Z1, Z0, Z1};
    MF_HIP(launch_value_forward_act(net, desc->width, ACT_GELU, C, X, x_per_bc, n_pts, n_bc * n_pts, Z, s));
    MF_HIP(launch_rows_output(net, desc->width, MF_CROSS, Z1, n_bc * n_pts, 0, U, 0, 0, 0, 0, 0, s));
  } else {
    MF_HIP(launch_forward_rows(net, desc->width, prec, C, X, n_bc, n_pts, x_per_bc, U, s));
  }
  return ok();
}

static mf_status train_sizes(int64_t B, int64_t nd, int64_t nc) {
  if (B < 1 || nd < 1 || nc < 1) return fail(MF_ESHAPE, "B, nd and nc must be >= 1");
  if (B * nc > (1LL << 31) / 4) return fail(MF_ESHAPE, "B * nc too large");
  if (B * nd > (1LL << 31) / 4) return fail(MF_ESHAPE, "B * nd too large");
  return MF_OK;
}

mf_status sdnet_train_ws_size(const mf_sdnet_desc* desc, int64_t B, int64_t nd, int64_t nc, size_t* bytes) {
  MF_TRY(check_ptr(bytes, "bytes", 1));
  *bytes = 0;
  MF_TRY(check_desc(desc));
  MF_TRY(train_sizes(B, nd, nc));
  *bytes = train_layout(desc, B, nd, nc).total;
  return ok();
}

mf_status sdnet_train_step(mf_ctx* ctx, const mf_sdnet_desc* desc, float* params, float* m, float* v,
                           int64_t step, const mf_adam* hp, const float* G, int64_t B, const float* Xd,
                           int64_t nd, int32_t xd_per_bc, const float* Yd, const float* Xc, int64_t nc,
                           float* loss_dev, float* grad_out, void* ws, size_t ws_bytes, void* stream) {
  MF_TRY(check_desc(desc));
  MF_TRY(train_sizes(B, nd, nc));
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(G, "G"));
  MF_TRY(check_ptr(Xd, "Xd"));
  MF_TRY(check_ptr(Xc, "Xc"));
  MF_TRY(check_ptr(loss_dev, "loss_dev"));
  if (xd_per_bc != 0 && xd_per_bc != 1) return fail(MF_EINVAL, "xd_per_bc %d is not 0 or 1", xd_per_bc);
  if (Yd) {
    MF_TRY(check_ptr(Yd, "Yd"));
  } else if (nd != 128) {
    return fail(MF_ESHAPE, "without Yd the targets are G, so nd must be 128 (got %lld)", (long long)nd);
  }
  if (grad_out) {
    MF_TRY(check_ptr(grad_out, "grad_out"));
  } else {
    MF_TRY(check_ptr(m, "m"));
    MF_TRY(check_ptr(v, "v"));
    if (!hp) return fail(MF_EINVAL, "adam hyperparameters are NULL");
    if (step < 1) return fail(MF_EINVAL, "step %lld < 1 (Adam counts from 1)", (long long)step);
    if (!(hp->lr > 0.0) || !(hp->beta1 >= 0.0 && hp->beta1 < 1.0) ||
        !(hp->beta2 >= 0.0 && hp->beta2 < 1.0) || !(hp->eps > 0.0))
      return fail(MF_EINVAL, "adam hyperparameters out of range");
  }
  const TrainLayout L = train_layout(desc, B, nd, nc);
  MF_TRY(check_ws(ws, ws_bytes, L.total));
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(prepare_net(desc, params, MF_FP32, L.net, ws, s));
  const NetPtrs net = net_ptrs(L.net, ws);
  // where the tensors sit: [convolutions] | W1 | b1 | W2 | b2 | W3 | b3 | W4 | b4 | w5 | b5
  TrainNet tn;
  tn.params = params;
  tn.channels = is_gelu(desc) ? desc->embed_channels : 0;
  tn.n_in = is_gelu(desc) ? 128 * desc->embed_channels : desc->n_boundary;
  const int64_t d = desc->width;
  tn.off_w1 = is_gelu(desc) ? embed_param_offset(desc->embed_channels) : 0;
  tn.off_w2 = tn.off_w1 + d * (tn.n_in + 2) + d;
  tn.off_w5 = tn.off_w2 + 3 * (d * d + d);
  float* whT = reinterpret_cast<float*>(static_cast<char*>(ws) + L.whT);
  MF_HIP(launch_prepare_wT(params, tn.off_w2, desc->width, whT, s));
  const TrainBuffers tb = train_buffers(L, ws);
  float* grad = grad_out ? grad_out : tb.grad;
  MF_HIP(launch_train_grad(tn, net, desc->width, whT, tb, G, B, Xd, nd, xd_per_bc, Yd, Xc, nc, grad, loss_dev, s));
  if (!grad_out)
    MF_HIP(launch_adam(params, m, v, grad, mf_param_count(desc), hp->lr, hp->beta1, hp->beta2, hp->eps,
                       step, s));
  return ok();
}

mf_status sdnet_loss_grad(mf_ctx* ctx, const mf_sdnet_desc* desc, const float* params, const float* G,
                          int64_t B, const float* Xd, int64_t nd, int32_t xd_per_bc, const float* Yd,
                          const float* Xc, int64_t nc, float* loss_dev, float* grad_out, void* ws,
                          size_t ws_bytes, void* stream) {
  MF_TRY(check_ptr(grad_out, "grad_out"));
  // the gradient mode of the training step reads params and updates nothing
  return sdnet_train_step(ctx, desc, const_cast<float*>(params), nullptr, nullptr, 1, nullptr, G, B, Xd, nd,
                          xd_per_bc, Yd, Xc, nc, loss_dev, grad_out, ws, ws_bytes, stream);
}

mf_status mf_param_segments(const mf_sdnet_desc* desc, int64_t* begin, int32_t capacity, int32_t* n_segments) {
  MF_TRY(check_desc(desc));
  if (!begin || !n_segments) return fail(MF_EINVAL, "begin or n_segments is NULL");
  const int64_t d = desc->width;
  int64_t sizes[16];
  int n = 0;
  int64_t in1 = desc->n_boundary;
  if (is_gelu(desc)) {   // conv 1 -> C and conv C -> C, kernel 5, each with its bias
    const int64_t C = desc->embed_channels;
    sizes[n++] = C * kConvK;
    sizes[n++] = C;
    sizes[n++] = C * C * kConvK;
    sizes[n++] = C;
    in1 = C * desc->n_boundary;
  }
  sizes[n++] = d * (in1 + 2);
  sizes[n++] = d;
  for (int l = 0; l < 3; ++l) {
    sizes[n++] = d * d;
    sizes[n++] = d;
  }
  sizes[n++] = d;
  sizes[n++] = 1;
  *n_segments = n;
  if (capacity < n) return fail(MF_ESHAPE, "capacity %d < %d tensors", capacity, n);
  begin[0] = 0;
  for (int i = 0; i < n; ++i) begin[i + 1] = begin[i] + sizes[i];
  if (begin[n] != mf_param_count(desc)) return fail(MF_EINVAL, "tensor table does not cover the parameters");
  return ok();
}

mf_status sdnet_lamb_step(mf_ctx* ctx, float* params, float* m, float* v, const float* grad,
                          const int64_t* seg_begin, int32_t n_segments, int64_t step, const mf_lamb* hp,
                          void* stream) {
  MF_TRY(check_ptr(params, "params"));
  MF_TRY(check_ptr(m, "m"));
  MF_TRY(check_ptr(v, "v"));
  MF_TRY(check_ptr(grad, "grad"));
  if (!seg_begin) return fail(MF_EINVAL, "seg_begin is NULL");
  if (n_segments < 1 || n_segments > MF_MAX_SEGMENTS)
    return fail(MF_EINVAL, "n_segments %d not in 1..%d", n_segments, (int)MF_MAX_SEGMENTS);
  if (seg_begin[0] != 0) return fail(MF_EINVAL, "seg_begin[0] must be 0");
  for (int i = 0; i < n_segments; ++i)
    if (seg_begin[i + 1] < seg_begin[i]) return fail(MF_EINVAL, "seg_begin decreases at %d", i + 1);
  if (seg_begin[n_segments] < 1) return fail(MF_EINVAL, "no parameters");
  if (!hp) return fail(MF_EINVAL, "lamb hyperparameters are NULL");
  if (step < 1) return fail(MF_EINVAL, "step %lld < 1 (LAMB counts from 1)", (long long)step);
  if (!(hp->lr >= 0.0) || !(hp->beta1 >= 0.0 && hp->beta1 < 1.0) || !(hp->beta2 >= 0.0 && hp->beta2 < 1.0) ||
      !(hp->eps >= 0.0) || !(hp->weight_decay >= 0.0) || !(hp->max_grad_norm >= 0.0))
    return fail(MF_EINVAL, "lamb hyperparameters out of range");
  if (hp->trust_without_decay != 0 && hp->trust_without_decay != 1)
    return fail(MF_EINVAL, "trust_without_decay %d is not 0 or 1", hp->trust_without_decay);
  if (!ctx) return fail(MF_EINVAL, "ctx is NULL");
  LambSegments S;
  S.n = n_segments;
  for (int i = 0; i <= n_segments; ++i) S.begin[i] = seg_begin[i];
  hipStream_t s = static_cast<hipStream_t>(stream);
  MF_HIP(hipSetDevice(ctx->device));
  MF_HIP(launch_lamb(params, m, v, grad, S, hp->lr, hp->beta1, hp->beta2, hp->eps, hp->weight_decay,
                     hp->max_grad_norm, hp->trust_without_decay == 1 || hp->weight_decay != 0.0, step, s));
  return ok();
}

static mf_status check_schedule(const mf_lr_schedule* sc) {
  if (!sc) return fail(MF_EINVAL, "schedule is NULL");
  if (sc->total_steps < 1) return fail(MF_EINVAL, "total_steps %lld < 1", (long long)sc->total_steps);
  if (!(sc->warmup_frac >= 0.0 && sc->warmup_frac <= 1.0)) return fail(MF_EINVAL, "warmup_frac not in [0, 1]");
  if (!(sc->max_lr >= 0.0) || !(sc->end_lr >= 0.0)) return fail(MF_EINVAL, "learning rates must be >= 0");
  if (!(sc->power > 0.0)) return fail(MF_EINVAL, "power must be > 0");
  return MF_OK;
}

mf_status mf_lr_at(const mf_lr_schedule* sc, int64_t step, double* lr) {
  MF_TRY(check_schedule(sc));
  if (!lr) return fail(MF_EINVAL, "lr is NULL");
  if (step < 1) return fail(MF_EINVAL, "step %lld < 1", (long long)step);
  const int64_t T = sc->total_steps;
  const int64_t W = (int64_t)ceil(sc->warmup_frac * (double)T);
  if (step <= W) {
    *lr = sc->max_lr * (double)step / (double)W;
  } else if (step >= T) {
    *lr = sc->end_lr;
  } else {
    const double frac = 1.0 - (double)(step - W) / (double)(T - W);
    *lr = sc->end_lr + (sc->max_lr - sc->end_lr) * pow(frac, sc->power);
  }
  return ok();
}

mf_status mf_lr_schedule_scaled(const mf_lr_schedule* base, double batch_factor, mf_lr_schedule* out) {
  MF_TRY(check_schedule(base));
  if (!out) return fail(MF_EINVAL, "out is NULL");
  if (!(batch_factor > 0.0)) return fail(MF_EINVAL, "batch_factor must be > 0");
  *out = *base;
  out->max_lr = base->max_lr * sqrt(batch_factor);
  out->warmup_frac = std::min(1.0, base->warmup_frac * batch_factor);
  return ok();
}

}  // extern "C"
