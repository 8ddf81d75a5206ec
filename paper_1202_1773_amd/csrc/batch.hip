// batch.hip -- uneven batches: images of several sizes transformed by one
// graph launch per direction (host code only; the kernels are the plans').
//
// Images of equal (M, N, J) form a class with one plan; every class runs the
// plan's batched passes on a stream of its own, forked from a capture stream
// by an event and joined back by one event per class. The whole fork/join is
// captured into a HIP graph, instantiated once per (input, output, workspace)
// triple (the eight most recently used triples per direction are kept) and
// launched on the caller's stream; the classes' kernels can then run side by
// side on the GPU with no host work between them.
#include "../../include/ffst.h"
#include "internal.hpp"
#include "launch_cfg.hpp"

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

using namespace ffst;

namespace {

constexpr unsigned kBatchMagic = 0x46464254u;  // "FFBT"
// Executable graphs kept per direction: callers that let the binding
// allocate a fresh output per call (or alternate between a few buffers)
// replay graphs instead of capturing one per call.
constexpr size_t kGraphsPerDirection = 8;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct ffst_batch {
  int count = 0;
  bool cplx = false;
  std::vector<ffst_plan*> plans;            // one per class
  std::vector<int> cls_images;              // images per class
  std::vector<long long> cls_img_off;       // float offsets of the class blocks
  std::vector<long long> cls_coef_off;
  std::vector<size_t> cls_ws_off, cls_ws_size;
  std::vector<long long> img_off, coef_off; // per image, in the caller's order
  long long img_total = 0, coef_total = 0;
  size_t ws_total = 0;
  int device = -1;
  hipStream_t capture = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  struct Graph {
    hipGraphExec_t exec = nullptr;
    const void* in = nullptr;
    const void* out = nullptr;
    const void* ws = nullptr;
    unsigned long long last_use = 0;
  };
  // per direction (0: forward, 1: adjoint), the executable graphs of the
  // most recently used (input, output, workspace) triples
  std::vector<Graph> graphs[2];
  unsigned long long uses = 0;
  unsigned magic = 0;
};

namespace {

bool batch_ok(const ffst_batch* b) { return b && b->magic == kBatchMagic; }

void drop_graphs(ffst_batch* b) {
  for (auto& dir : b->graphs) {
    for (auto& g : dir)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    dir.clear();
  }
}

void free_batch(ffst_batch* b) {
  if (!b) return;
  drop_graphs(b);
  for (auto* p : b->plans) ffst_destroy(p);
  for (auto s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  for (auto e : b->joins)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  b->magic = 0;
  delete b;
}

int plan_eta(const ffst_plan* p) {
  int eta = 0;
  ffst_plan_info(p, nullptr, nullptr, nullptr, &eta);
  return eta;
}

void plan_size(const ffst_plan* p, int* M, int* N) { ffst_plan_info(p, M, N, nullptr, nullptr); }

// Records the launches of one direction for every class, fork/join around
// the capture stream, into a new executable graph.
int capture(ffst_batch* b, int dir, const float* in, float* out, void* ws, hipGraphExec_t* exec) {
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return fail(FFST_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  profile_suspend(true);
  int st = FFST_OK;
  if ((e = hipEventRecord(b->fork, b->capture)) != hipSuccess)
    st = fail(FFST_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  const size_t nc = b->plans.size();
  for (size_t c = 0; c < nc && st == FFST_OK; ++c) {
    hipStream_t s = b->streams[c];
    if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) {
      st = fail(FFST_EDEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
      break;
    }
    void* cws = static_cast<char*>(ws) + b->cls_ws_off[c];
    const ffst_plan* p = b->plans[c];
    if (dir == 0) {
      const float* f = in + b->cls_img_off[c];
      float* co = out + b->cls_coef_off[c];
      st = b->cplx ? ffst_forward_complex(p, f, co, b->cls_images[c], cws, s)
                   : ffst_forward(p, f, co, b->cls_images[c], cws, s);
    } else {
      const float* co = in + b->cls_coef_off[c];
      float* f = out + b->cls_img_off[c];
      st = b->cplx ? ffst_adjoint_complex(p, co, f, b->cls_images[c], cws, s)
                   : ffst_adjoint(p, co, f, b->cls_images[c], cws, s);
    }
    if (st == FFST_OK && (e = hipEventRecord(b->joins[c], s)) != hipSuccess)
      st = fail(FFST_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    if (st == FFST_OK && (e = hipStreamWaitEvent(b->capture, b->joins[c], 0)) != hipSuccess)
      st = fail(FFST_EDEVICE, "hipStreamWaitEvent: %s", hipGetErrorString(e));
  }
  profile_suspend(false);
  // the capture is always ended, also after a failure, so the stream leaves capture mode
  e = hipStreamEndCapture(b->capture, &graph);
  if (st == FFST_OK && e != hipSuccess) st = fail(FFST_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  if (st == FFST_OK && (e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0)) != hipSuccess)
    st = fail(FFST_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  if (graph) (void)hipGraphDestroy(graph);
  return st;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

int run(ffst_batch* b, int dir, const float* in, float* out, void* ws, void* stream, const char* what) {
  const Range range(what);
  if (!batch_ok(b)) return fail(FFST_EBADPLAN, "%s: invalid batch", what);
  if (!in || !out || !ws) return fail(FFST_EINVAL, "%s: buffers must be non-NULL", what);
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(FFST_EINVAL, "%s: workspace must be 256-byte aligned", what);
  if (reinterpret_cast<uintptr_t>(in) % 8 || reinterpret_cast<uintptr_t>(out) % 8)
    return fail(FFST_EINVAL, "%s: input and output must be 8-byte aligned", what);
  const size_t img_bytes = (size_t)b->img_total * sizeof(float), coef_bytes = (size_t)b->coef_total * sizeof(float);
  const size_t in_bytes = dir == 0 ? img_bytes : coef_bytes, out_bytes = dir == 0 ? coef_bytes : img_bytes;
  if (overlaps(in, in_bytes, out, out_bytes) || overlaps(ws, b->ws_total, in, in_bytes) ||
      overlaps(ws, b->ws_total, out, out_bytes))
    return fail(FFST_EINVAL, "%s: input, output and workspace must not overlap", what);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return fail(FFST_EINVAL, "%s: the current device is not the batch's device %d", what, b->device);
  std::vector<ffst_batch::Graph>& cache = b->graphs[dir];
  ffst_batch::Graph* g = nullptr;
  for (auto& c : cache)
    if (c.in == in && c.out == out && c.ws == ws) g = &c;
  if (!g) {
    hipGraphExec_t exec = nullptr;
    const int st = capture(b, dir, in, out, ws, &exec);
    if (st != FFST_OK) return st;
    if (cache.size() >= kGraphsPerDirection) {  // replace the least recently used
      auto lru = std::min_element(cache.begin(), cache.end(), [](const ffst_batch::Graph& x,
                                                                 const ffst_batch::Graph& y) {
        return x.last_use < y.last_use;
      });
      (void)hipGraphExecDestroy(lru->exec);
      *lru = ffst_batch::Graph{exec, in, out, ws, 0};
      g = &*lru;
    } else {
      cache.push_back(ffst_batch::Graph{exec, in, out, ws, 0});
      g = &cache.back();
    }
  }
  g->last_use = ++b->uses;
  const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(FFST_EDEVICE, "%s: hipGraphLaunch: %s", what, hipGetErrorString(e));
  return FFST_OK;
}

// Forward + adjoint of the whole batch through its graphs: the best of 3
// runs after one warm-up, HIP events on `stream`.
int time_batch(ffst_batch* b, const float* f, float* coeffs, float* out, void* ws, void* stream, double* best_ms) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(FFST_EDEVICE, "ffst_batch_tune: hipEventCreate failed");
  }
  int st = FFST_OK;
  double best = -1.0;
  for (int rep = 0; rep < 4 && st == FFST_OK; ++rep) {
    (void)hipEventRecord(e0, s);
    st = run(b, 0, f, coeffs, ws, stream, "ffst_batch_tune");
    if (st == FFST_OK) st = run(b, 1, coeffs, out, ws, stream, "ffst_batch_tune");
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (st == FFST_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(FFST_EDEVICE, "ffst_batch_tune: event timing failed");
    if (st == FFST_OK && rep > 0 && (best < 0 || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ms = best;
  return st;
}

}  // namespace

extern "C" {

int ffst_batch_create(int count, const int* M, const int* N, const int* J, const ffst_options* opt,
                      ffst_batch** out) {
  const Range range("ffst_batch_create");
  const AllocScope alloc_scope;
  if (!out) return fail(FFST_EINVAL, "out must be non-NULL");
  *out = nullptr;
  if (count < 1) return fail(FFST_EINVAL, "count must be >= 1 (got %d)", count);
  if (!M || !N || !J) return fail(FFST_EINVAL, "size arrays must be non-NULL");
  ffst_batch* b = new (std::nothrow) ffst_batch();
  if (!b) return fail(FFST_ENOMEM, "host allocation failed");
  b->magic = kBatchMagic;
  b->count = count;
  b->cplx = opt && opt->complex_shearlets == 1;
  if (hipGetDevice(&b->device) != hipSuccess) {
    free_batch(b);
    return fail(FFST_EDEVICE, "hipGetDevice failed");
  }
  (void)num_cus();  // device query done here, not while a graph is captured
  // classes in the order of their first image
  std::map<std::tuple<int, int, int>, int> index;
  std::vector<int> cls_of(count);
  for (int i = 0; i < count; ++i) {
    ffst_plan* probe = nullptr;
    const auto key = std::make_tuple(M[i], N[i], J[i]);
    auto it = index.find(key);
    if (it == index.end()) {
      const int st = ffst_spectra_ex(M[i], N[i], J[i], opt, &probe);
      if (st != FFST_OK) {
        free_batch(b);
        return st;  // message set by ffst_spectra_ex
      }
      it = index.emplace(key, (int)b->plans.size()).first;
      b->plans.push_back(probe);
      b->cls_images.push_back(0);
    }
    cls_of[i] = it->second;
    b->cls_images[it->second] += 1;
  }
  const size_t nc = b->plans.size();
  const long long cmul = b->cplx ? 2 : 1;
  b->cls_img_off.resize(nc);
  b->cls_coef_off.resize(nc);
  b->cls_ws_off.resize(nc);
  b->cls_ws_size.resize(nc);
  long long io = 0, co = 0;
  size_t wo = 0;
  // class blocks start on 256-byte boundaries (64 floats): images of odd
  // size would otherwise leave the next class misaligned for its plan
  auto align64 = [](long long x) { return (x + 63) & ~63LL; };
  for (size_t c = 0; c < nc; ++c) {
    int m = 0, n = 0;
    plan_size(b->plans[c], &m, &n);
    const long long mn = (long long)m * n;
    b->cls_img_off[c] = io;
    b->cls_coef_off[c] = co;
    io = align64(io + mn * b->cls_images[c]);
    co = align64(co + cmul * plan_eta(b->plans[c]) * mn * b->cls_images[c]);
    b->cls_ws_off[c] = wo;
    b->cls_ws_size[c] = align256(workspace_upper_bound(b->plans[c], b->cls_images[c]));
    wo += b->cls_ws_size[c];
  }
  b->img_total = io;
  b->coef_total = co;
  b->ws_total = std::max<size_t>(wo, 256);
  b->img_off.resize(count);
  b->coef_off.resize(count);
  std::vector<int> seen(nc, 0);
  for (int i = 0; i < count; ++i) {
    const int c = cls_of[i];
    int m = 0, n = 0;
    plan_size(b->plans[c], &m, &n);
    const long long mn = (long long)m * n;
    b->img_off[i] = b->cls_img_off[c] + mn * seen[c];
    b->coef_off[i] = b->cls_coef_off[c] + cmul * plan_eta(b->plans[c]) * mn * seen[c];
    seen[c] += 1;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  b->streams.assign(nc, nullptr);
  b->joins.assign(nc, nullptr);
  for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&b->streams[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->joins[c], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    free_batch(b);
    return fail(FFST_EDEVICE, "stream/event creation: %s", hipGetErrorString(e));
  }
  *out = b;
  log_line(1, "batch %p: %d image(s) in %zu size class(es), %lld coefficients, workspace %zu bytes", (void*)b, count, nc,
       (long long)b->coef_total, b->ws_total);
  for (size_t c = 0; c < nc; ++c) {
    int cm = 0, cn = 0, cj = 0;
    (void)ffst_plan_info(b->plans[c], &cm, &cn, &cj, nullptr);
    log_line(1, "batch %p class %zu: %d image(s) of %d x %d, J = %d, plan %p", (void*)b, c, b->cls_images[c], cm, cn, cj,
         (void*)b->plans[c]);
  }
  return FFST_OK;
}

int ffst_batch_info(const ffst_batch* b, int* count, int* classes) {
  if (!batch_ok(b)) return fail(FFST_EBADPLAN, "invalid batch");
  if (count) *count = b->count;
  if (classes) *classes = (int)b->plans.size();
  return FFST_OK;
}

int ffst_batch_class(const ffst_batch* b, int cls, ffst_plan** plan, int* images) {
  if (!batch_ok(b)) return fail(FFST_EBADPLAN, "invalid batch");
  if (cls < 0 || cls >= (int)b->plans.size()) return fail(FFST_EINVAL, "class %d out of range", cls);
  if (plan) *plan = b->plans[cls];
  if (images) *images = b->cls_images[cls];
  return FFST_OK;
}

int ffst_batch_layout(const ffst_batch* b, long long* img_offset, long long* coef_offset, long long* img_total,
                      long long* coef_total) {
  if (!batch_ok(b)) return fail(FFST_EBADPLAN, "invalid batch");
  if (img_offset) std::copy(b->img_off.begin(), b->img_off.end(), img_offset);
  if (coef_offset) std::copy(b->coef_off.begin(), b->coef_off.end(), coef_offset);
  if (img_total) *img_total = b->img_total;
  if (coef_total) *coef_total = b->coef_total;
  return FFST_OK;
}

size_t ffst_batch_workspace_size(const ffst_batch* b) { return batch_ok(b) ? b->ws_total : 0; }

int ffst_batch_forward(ffst_batch* b, const float* f, float* coeffs, void* ws, void* stream) {
  return run(b, 0, f, coeffs, ws, stream, "ffst_batch_forward");
}

int ffst_batch_adjoint(ffst_batch* b, const float* coeffs, float* f, void* ws, void* stream) {
  return run(b, 1, coeffs, f, ws, stream, "ffst_batch_adjoint");
}

int ffst_batch_inverse(ffst_batch* b, const float* coeffs, float* f, void* ws, void* stream) {
  return run(b, 1, coeffs, f, ws, stream, "ffst_batch_inverse");
}

int ffst_batch_tune(ffst_batch* b, const float* f, float* coeffs, float* out, void* ws, void* stream) {
  const Range range("ffst_batch_tune");
  if (!batch_ok(b)) return fail(FFST_EBADPLAN, "invalid batch");
  if (!f || !coeffs || !out || !ws) return fail(FFST_EINVAL, "ffst_batch_tune: buffers must be non-NULL");
  // Every class is tuned on its own; the classes then run side by side, so
  // the tuned settings are kept only if the whole batch is faster with them.
  const size_t nc = b->plans.size();
  std::vector<ffst_tuning> saved(nc);
  for (size_t c = 0; c < nc; ++c) ffst_get_tuning_ex(b->plans[c], &saved[c]);
  double before = 0.0, after = 0.0;
  int st = time_batch(b, f, coeffs, out, ws, stream, &before);
  drop_graphs(b);
  for (size_t c = 0; c < nc && st == FFST_OK; ++c)
    st = ffst_tune(b->plans[c], f + b->cls_img_off[c], coeffs + b->cls_coef_off[c], out + b->cls_img_off[c],
                   b->cls_images[c], static_cast<char*>(ws) + b->cls_ws_off[c], b->cls_ws_size[c], stream, nullptr);
  drop_graphs(b);
  if (st == FFST_OK) st = time_batch(b, f, coeffs, out, ws, stream, &after);
  if (st != FFST_OK || after > before) {
    for (size_t c = 0; c < nc; ++c) ffst_set_tuning_ex(b->plans[c], &saved[c]);
    drop_graphs(b);
  }
  if (st == FFST_OK)
    log_line(1, "batch %p tuned: %.4f ms before, %.4f ms with the classes' own settings; %s", (void*)b, before, after,
         after > before ? "kept the previous settings" : "kept the tuned settings");
  return st;
}

void ffst_batch_destroy(ffst_batch* b) {
  if (!batch_ok(b)) return;
  log_line(1, "batch %p destroyed", (void*)b);
  (void)hipDeviceSynchronize();
  free_batch(b);
}

}  // extern "C"
