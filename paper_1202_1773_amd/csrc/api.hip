// api.hip -- plan management and the C ABI declared in include/ffst.h.
#include "../../include/ffst.h"
#include "internal.hpp"
#include "launch_cfg.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

using namespace ffst;

struct ffst_plan {
  int M = 0, N = 0, J = 0, eta = 0, H = 0;
  int pitch = 0;                // complex elements between column lines of the complex buffers
  int device = -1;
  ffst_options opt{};
  double delta = 0.0;
  // device buffers owned by the plan
  float* psi = nullptr;         // [eta][H][M] (column-contiguous)
  float2* twM = nullptr;        // exp(-2 pi i m / M), m < M
  float2* twN = nullptr;        // exp(-2 pi i m / N), m < N
  int* d_lo = nullptr;          // per-plane window start, width, offset
  int* d_w = nullptr;
  long long* d_off = nullptr;
  int* d_img_lo = nullptr;      // single full window for image-sized passes
  int* d_img_w = nullptr;
  long long* d_img_off = nullptr;
  // every window column line of Psi_i (real) or Psi+_i (complex) over its
  // cyclic nonzero hull (see FwdColArgs), for the CSR entries of both column
  // passes
  float* psic = nullptr;
  int4* d_col_hull = nullptr;
  int* d_col_ptr = nullptr;     // per plane group: columns -> spectra (CSR, absolute pointers)
  int* d_col_planes = nullptr;
  // complex shearlets: compact one-sided spectra over cyclic full-plane
  // windows (kept for ffst_get_spectra)
  float* psip = nullptr;        // plane i: w[i] columns of M values at psip + poff[i]
  long long* d_poff = nullptr;
  int2* d_col_ent = nullptr;    // forward CSR entries (spectrum, 4 * window column + flags)
  int* d_acol_ptr = nullptr;    // adjoint CSR (complex): columns -> entries with flag 1 or 2,
  int2* d_acol_ent = nullptr;   //   hulls of the reversed lines for flag 2
  int4* d_acol_hull = nullptr;
  // host copies
  std::vector<int> lo, w;
  std::vector<long long> off;
  std::vector<long long> poff;
  long long zimg = 0;           // complex elements of one image's compact buffer
  std::vector<int> groups;      // plane-group boundaries p0 < p1 < ... (ngroups + 1)
  long long chunk_elems = 0;    // target size of one unit's compact buffer
  int tune_nparts = 0;          // lines per column in the adjoint column pass (0: heuristic)
  int tune_fwd_nparts = 0;      // lines per column in the forward column pass (0: heuristic)
  int tune_blocks_per_cu = 0;   // persistent blocks per CU (0: per-kernel default)
  int tune_col_values = 0;      // values per lane of the column-line FFTs (0: default)
  int tune_row_block = 0;       // row blocks of the row kernels (0/1: default height, 2: the alternative)
  unsigned magic = 0;
};

namespace {
thread_local std::string g_err;
}  // namespace

int ffst::fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  log_line(1, "error %d: %s", status, buf);
  return status;
}

// ---- device memory held by plans and batches ---------------------------
//
// Every device allocation of the library goes through dev_alloc / dev_free,
// which keep the bytes held (ffst_device_bytes) and let a test make the n-th
// allocation of one plan or batch creation fail: with FFST_FAULT_ALLOC=n in
// the environment, the n-th dev_alloc inside one ffst_spectra_ex or
// ffst_batch_create call (nested calls count towards the outer one) returns
// hipErrorOutOfMemory without allocating, so every cleanup path can be run.
namespace {
std::mutex g_mem_mu;
std::unordered_map<void*, size_t> g_live;
std::atomic<size_t> g_live_bytes{0};
thread_local int t_alloc_depth = 0;
thread_local int t_alloc_calls = 0;

int fault_alloc_index() {
  const char* v = std::getenv("FFST_FAULT_ALLOC");
  return v ? std::atoi(v) : 0;
}
}  // namespace

ffst::AllocScope::AllocScope() {
  if (t_alloc_depth++ == 0) t_alloc_calls = 0;
}
ffst::AllocScope::~AllocScope() { --t_alloc_depth; }

hipError_t ffst::dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  const int fail_at = fault_alloc_index();
  if (fail_at > 0 && ++t_alloc_calls == fail_at) return hipErrorOutOfMemory;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  std::lock_guard<std::mutex> lk(g_mem_mu);
  g_live[*p] = bytes;
  g_live_bytes += bytes;
  return hipSuccess;
}

void ffst::dev_free(void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_mem_mu);
    auto it = g_live.find(p);
    if (it != g_live.end()) {
      g_live_bytes -= it->second;
      g_live.erase(it);
    }
  }
  (void)hipFree(p);
}

namespace {

constexpr unsigned kMagic = 0x46465354u;  // "FFST"

int ok() { return FFST_OK; }

bool plan_ok(const ffst_plan* p) { return p && p->magic == kMagic; }

// ---- kernel timing -----------------------------------------------------
const char* kKernelNames[KID_COUNT] = {
    "k_spectra", "k_windows", "k_r2c_rows(image)", "k_fwd_cols",
    "k_c2r_rows(planes)", "k_r2c_rows(planes)", "k_adj_cols", "k_col_fft(inverse)",
    "k_c2r_rows(image)", "k_expand", "k_one_sided", "k_fwd_cols(complex)", "k_c2c_rows(planes, inverse)",
    "k_c2c_rows(planes)", "k_adj_cols(complex)"};

struct ProfRec {
  int id;
  hipEvent_t a, b;
};
// Read by every transform call, on any thread: atomics (relaxed; the
// timing records themselves are not thread-safe).
std::atomic<unsigned> g_mask{0};
std::atomic<bool> g_profile_suspended{false};  // set while a graph is being captured
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;  // events reused across timed launches
double g_total_ms[KID_COUNT] = {};
long long g_count[KID_COUNT] = {};

hipEvent_t pooled_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Set for the duration of a call that must not create HIP objects (events).
thread_local bool t_no_timing = false;
// Set while the autotuner runs its candidates (their calls are not logged).
thread_local bool t_tuning_calls = false;

template <class Fn>
hipError_t timed(int id, hipStream_t s, Fn&& fn) {
  const Range range(kKernelNames[id]);
  if (t_no_timing || g_profile_suspended.load(std::memory_order_relaxed) ||
      !((g_mask.load(std::memory_order_relaxed) >> id) & 1u))
    return fn();
  ProfRec r{id, pooled_event(), pooled_event()};
  if (!r.a || !r.b) return fn();
  (void)hipEventRecord(r.a, s);
  hipError_t e = fn();
  (void)hipEventRecord(r.b, s);
  g_recs.push_back(r);
  return e;
}

void drain_profile() {
  for (auto& r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_total_ms[r.id] += ms;
      g_count[r.id] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

// ---- plan construction -------------------------------------------------


int default_scales(int M, int N) {
  int L = std::max(M, N), lg = 0;
  while ((L >> (lg + 1)) > 0) ++lg;  // floor(log2 L)
  return lg / 2;
}

// Index order of Sec. 3.5.2: per scale h k = 0, -1 .. -2^j+1; seam -2^j;
// v -2^j+1 .. 2^j-1; seam 2^j; h 2^j-1 .. 1. Low-pass first.
void index_order(int J, std::vector<int>& kind, std::vector<int>& jj, std::vector<int>& kk) {
  kind = {KIND_LOWPASS};
  jj = {0};
  kk = {0};
  auto push = [&](int kd, int j, int k) {
    kind.push_back(kd);
    jj.push_back(j);
    kk.push_back(k);
  };
  for (int j = 0; j < J; ++j) {
    const int P = 1 << j;
    for (int k = 0; k > -P; --k) push(KIND_H, j, k);
    push(KIND_SEAM, j, -P);
    for (int k = -P + 1; k < P; ++k) push(KIND_V, j, k);
    push(KIND_SEAM, j, P);
    for (int k = P - 1; k > 0; --k) push(KIND_H, j, k);
  }
}

std::vector<float2> twiddles(int L) {
  std::vector<float2> t(L);
  for (int m = 0; m < L; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)L;
    t[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return t;
}

// Frees device memory whose release status no caller can act on.
void release(void* ptr) { dev_free(ptr); }

void release_event(hipEvent_t e) {
  if (e) (void)hipEventDestroy(e);
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  hipError_t e = dev_alloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

void free_plan(ffst_plan* p) {
  if (!p) return;
  void* bufs[] = {p->psi, p->twM, p->twN, p->d_lo, p->d_w, p->d_off, p->d_img_lo, p->d_img_w,
                  p->d_img_off, p->d_col_ptr, p->d_col_planes, p->psip, p->d_poff, p->d_col_ent,
                  p->psic, p->d_col_hull, p->d_acol_ptr, p->d_acol_ent, p->d_acol_hull};
  for (void* b : bufs)
    if (b) release(b);
  p->magic = 0;
  delete p;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// How a call with `batch` images is cut into units of (images, plane group)
// whose compact intermediate stays near the target size, and how the
// adjoint's sum over spectra is spread over blocks.
struct Schedule {
  int chunk_imgs = 1;     // images per unit
  int nparts = 1;         // lines per (image, column) in the adjoint column pass (partial sums)
  int fwd_nparts = 1;     // lines per (image, column) in the forward column pass
  bool fused = true;      // adjoint column pass ends with its inverse FFT
  size_t fa_bytes = 0, yz_bytes = 0, part_bytes = 0;
};

Schedule schedule(const ffst_plan* p, int batch) {
  Schedule sc;
  const int ngroups = (int)p->groups.size() - 1;
  long long max_group = 0;
  for (int g = 0; g < ngroups; ++g)
    max_group = std::max(max_group, p->off[p->groups[g + 1] - 1] + (long long)p->pitch * p->w[p->groups[g + 1] - 1] -
                                        p->off[p->groups[g]]);
  if (ngroups == 1 && p->zimg > 0)
    sc.chunk_imgs = (int)std::max(1LL, std::min<long long>(batch, p->chunk_elems / std::max(1LL, p->zimg)));
  // row kernels index rows and images with 32-bit integers
  const long long rows_per_img = (long long)p->eta * p->M;
  sc.chunk_imgs = (int)std::max(1LL, std::min<long long>(sc.chunk_imgs, (1LL << 30) / rows_per_img));
  // and recover (image, plane) from a float reciprocal, exact below 2^20 planes
  sc.chunk_imgs = std::max(1, std::min(sc.chunk_imgs, (1 << 20) / p->eta));
  sc.chunk_imgs = std::max(1, std::min(sc.chunk_imgs, std::max(batch, 1)));
  // adjoint column lines per unit; below ~2 lines per SIMD the spectra of a
  // column are split over several lines (partial sums)
  const long long units = (long long)p->H * sc.chunk_imgs;
  const long long want = 8LL * 256;
  sc.nparts = (int)std::min<long long>(8, std::max<long long>(1, (want + units - 1) / units));
  if (p->tune_nparts > 0) sc.nparts = p->tune_nparts;
  sc.fused = (ngroups == 1 && sc.nparts == 1);
  // forward column lines: every line repeats the column's FFT of the image
  // spectrum, no partial sums, so it is split further (~8 lines per SIMD)
  const long long want_fwd = 32LL * 256;
  sc.fwd_nparts = (int)std::min<long long>(8, std::max<long long>(1, (want_fwd + units - 1) / units));
  if (p->tune_fwd_nparts > 0) sc.fwd_nparts = p->tune_fwd_nparts;
  sc.fa_bytes = align256((size_t)batch * p->pitch * p->H * sizeof(float2));
  sc.yz_bytes = align256((size_t)sc.chunk_imgs * (size_t)max_group * sizeof(float2));
  sc.part_bytes = sc.fused ? 0 : align256((size_t)sc.nparts * sc.chunk_imgs * p->pitch * p->H * sizeof(float2));
  return sc;
}

size_t ws_bytes(const ffst_plan* p, int batch) {
  if (batch <= 0) return 0;
  const Schedule sc = schedule(p, batch);
  return sc.fa_bytes + sc.yz_bytes + sc.part_bytes;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

int check_call(const ffst_plan* p, const void* in, size_t in_bytes, const void* out, size_t out_bytes,
               int batch, const void* ws) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (batch < 0) return fail(FFST_EINVAL, "batch must be >= 0 (got %d)", batch);
  if (batch == 0) return FFST_OK;
  if (!in || !out) return fail(FFST_EINVAL, "input and output must be non-NULL");
  if (!ws) return fail(FFST_EINVAL, "workspace must be non-NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(FFST_EINVAL, "workspace must be 256-byte aligned");
  if (reinterpret_cast<uintptr_t>(in) % 8 || reinterpret_cast<uintptr_t>(out) % 8)
    return fail(FFST_EINVAL, "input and output must be 8-byte aligned");
  if (overlap(in, in_bytes, out, out_bytes)) return fail(FFST_EINVAL, "input and output overlap");
  const size_t wsb = ws_bytes(p, batch);
  if (overlap(ws, wsb, in, in_bytes) || overlap(ws, wsb, out, out_bytes))
    return fail(FFST_EINVAL, "workspace overlaps input or output");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFST_EDEVICE, "hipGetDevice failed");
  if (dev != p->device)
    return fail(FFST_EINVAL, "current device %d is not the plan's device %d", dev, p->device);
  return FFST_OK;
}

int launched(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(FFST_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return FFST_OK;
}

// Smallest cyclic range of columns holding every flagged column: the
// complement of the longest cyclic run of unflagged columns (the first such
// run on ties). w = 0 for no flagged column.
void cyclic_window(const unsigned char* f, int N, int* lo, int* w) {
  int best = -1, start = 0, nflag = 0;
  for (int c = 0; c < N; ++c) nflag += f[c] != 0;
  if (nflag == 0) {
    *lo = 0;
    *w = 0;
    return;
  }
  if (nflag == N) {
    *lo = 0;
    *w = N;
    return;
  }
  for (int s = 0; s < N; ++s) {
    if (f[s] || !f[(s + N - 1) % N]) continue;  // not the start of an unflagged run
    int len = 0;
    while (!f[(s + len) % N]) ++len;
    if (len > best) {
      best = len;
      start = s;
    }
  }
  *lo = (start + best) % N;
  *w = N - best;
}

// Complex shearlets: windows of the one-sided spectra from their column
// flags, then the compact float32 spectra (evaluated in float64). The half-
// plane real spectra are released afterwards.
hipError_t one_sided_spectra(ffst_plan* p, const GenParams& g, const int* d_kind, const int* d_j, const int* d_k) {
  const int M = p->M, N = p->N, eta = p->eta;
  unsigned char* d_flags = nullptr;
  hipError_t e = dev_alloc(reinterpret_cast<void**>(&d_flags), (size_t)eta * N);
  if (e != hipSuccess) return e;
  e = timed(KID_ONE_SIDED, nullptr,
            [&] { return launch_one_sided_flags(p->psi, M, N, eta, d_kind, d_j, d_k, d_flags, nullptr); });
  std::vector<unsigned char> flags((size_t)eta * N);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(flags.data(), d_flags, flags.size(), hipMemcpyDeviceToHost);
  release(d_flags);
  if (e != hipSuccess) return e;
  p->poff.assign(eta, 0);
  long long total = 0;
  int max_w = 0;
  for (int i = 0; i < eta; ++i) {
    cyclic_window(flags.data() + (size_t)i * N, N, &p->lo[i], &p->w[i]);
    p->poff[i] = total;
    total += (long long)p->w[i] * M;
    max_w = std::max(max_w, p->w[i]);
  }
  if ((e = upload(&p->d_lo, p->lo)) != hipSuccess || (e = upload(&p->d_w, p->w)) != hipSuccess ||
      (e = upload(&p->d_poff, p->poff)) != hipSuccess)
    return e;
  if ((e = dev_alloc(reinterpret_cast<void**>(&p->psip), (size_t)std::max(total, 1LL) * sizeof(float))) != hipSuccess)
    return e;
  e = timed(KID_ONE_SIDED, nullptr, [&] {
    return launch_one_sided_pack(g, eta, max_w, d_kind, d_j, d_k, p->d_lo, p->d_w, p->d_poff, p->psip, nullptr);
  });
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) {
    release(p->psi);
    p->psi = nullptr;
  }
  return e;
}

int reject_kind(const ffst_plan* p, bool want_complex, const char* call) {
  if (p->opt.complex_shearlets == (want_complex ? 1 : 0)) return FFST_OK;
  return fail(FFST_EINVAL, "%s: the plan has %s shearlets", call, want_complex ? "real" : "complex");
}

// Applies a plan's persistent-grid setting to the launches of one call.
struct TuningScope {
  int saved_b, saved_v, saved_r;
  explicit TuningScope(const ffst_plan* p)
      : saved_b(t_blocks_per_cu), saved_v(t_col_values), saved_r(t_row_block) {
    t_blocks_per_cu = p->tune_blocks_per_cu;
    t_col_values = p->tune_col_values;
    t_row_block = p->tune_row_block == 2 ? 2 : 1;
  }
  ~TuningScope() {
    t_blocks_per_cu = saved_b;
    t_col_values = saved_v;
    t_row_block = saved_r;
  }
};

// The launch shapes compiled for a plan's sizes besides the defaults.
int alt_col_values_of(const ffst_plan* p) { return alt_col_values(p->M); }
bool row_block_tunable_of(const ffst_plan* p) { return p->N % 2 == 0 && row_block_tunable(p->N / 2); }

// Smallest cyclic range [lo, lo + K) (mod M) holding every nonzero value of
// a column line: the complement of its longest cyclic run of zeros (the
// first such run on ties). K = 0 for an all-zero line.
void cyclic_hull(const float* col, int M, int* lo, int* K) {
  int first_nz = -1;
  for (int r = 0; r < M && first_nz < 0; ++r)
    if (col[r] != 0.f) first_nz = r;
  if (first_nz < 0) {
    *lo = 0;
    *K = 0;
    return;
  }
  // scan the rotation that starts at a nonzero value, so every zero run is
  // contiguous in the scan
  int best = 0, best_end = first_nz, run = 0;
  for (int m = 1; m <= M; ++m) {
    const int r = (first_nz + m) % M;
    if (m < M && col[r] == 0.f) {
      ++run;
    } else {
      if (run > best) {
        best = run;
        best_end = r;                 // first nonzero after the run
      }
      run = 0;
    }
  }
  *lo = best > 0 ? best_end : first_nz;
  *K = M - best;
}

// Column lines of M values (host copy) over their hulls: values appended to
// psic, one (r_lo, K, offset) per line appended to hull_of.
hipError_t line_hulls(const float* lines, long long nlines, int M, std::vector<float>& psic,
                      std::vector<int4>& hull_of) {
  for (long long l = 0; l < nlines; ++l) {
    const float* col = lines + l * M;
    int lo = 0, K = 0;
    cyclic_hull(col, M, &lo, &K);
    if (psic.size() + (size_t)K > (size_t)INT32_MAX) return hipErrorNotSupported;   // offsets would overflow
    hull_of.push_back(make_int4(lo, K, (int)psic.size(), 0));
    for (int k = 0; k < K; ++k) psic.push_back(col[(lo + k) % M]);
  }
  return hipSuccess;
}

// Psi_i over the hulls of its window column lines, in plane order: the line
// of window column m of plane i is hull_of[base[i] + m]. Real plans read the
// half-plane spectra, complex plans the one-sided ones (stored by window
// line already).
hipError_t spectrum_hulls(const ffst_plan* p, std::vector<float>& psic, std::vector<int4>& hull_of,
                          std::vector<long long>& base) {
  const int M = p->M;
  const bool cplx = p->opt.complex_shearlets == 1;
  base.assign(p->eta + 1, 0);
  for (int i = 0; i < p->eta; ++i) base[i + 1] = base[i] + p->w[i];
  std::vector<float> buf;
  hipError_t e = hipSuccess;
  if (cplx) {
    buf.resize((size_t)base[p->eta] * M);
    if (!buf.empty())
      e = hipMemcpy(buf.data(), p->psip, buf.size() * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = line_hulls(buf.data(), base[p->eta], M, psic, hull_of);
  } else {
    for (int i = 0; i < p->eta && e == hipSuccess; ++i) {
      if (p->w[i] == 0) continue;
      buf.resize((size_t)p->w[i] * M);
      e = hipMemcpy(buf.data(), p->psi + ((size_t)i * p->H + p->lo[i]) * M, buf.size() * sizeof(float),
                    hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = line_hulls(buf.data(), p->w[i], M, psic, hull_of);
    }
  }
  if (psic.empty()) psic.push_back(0.f);
  return e;
}

Windows plane_windows(const ffst_plan* p) { return Windows{p->d_lo, p->d_w, p->d_off}; }
Windows image_window(const ffst_plan* p) { return Windows{p->d_img_lo, p->d_img_w, p->d_img_off}; }

}  // namespace

void ffst::profile_suspend(bool on) { g_profile_suspended.store(on, std::memory_order_relaxed); }

// ---- static scratch for callers that cannot allocate -------------------
//
// ffst_forward_noalloc runs ffst_forward with its workspace in this
// file-scope device array instead of caller memory. Every GPU the library
// runs on holds its own copy for the life of the process. In host code the
// name `scratch` is only a host-side stand-in: its device address on the
// current device comes from hipGetSymbolAddress, looked up once per device
// (with that device current) and kept in g_scratch_ptr; only that pointer
// is handed to kernels.
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FFST_EUNSUPPORTED, "device %d beyond the static scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FFST_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FFST_OK;
}

struct NoTimingScope {
  bool saved;
  NoTimingScope() : saved(t_no_timing) { t_no_timing = true; }
  ~NoTimingScope() { t_no_timing = saved; }
};
}  // namespace

size_t ffst::workspace_upper_bound(const ffst_plan* p, int batch) {
  if (!plan_ok(p) || batch <= 0) return 0;
  ffst_plan* q = const_cast<ffst_plan*>(p);
  const int saved = q->tune_nparts;
  size_t most = 0;
  for (int n = 1; n <= 8; ++n) {
    q->tune_nparts = n;
    most = std::max(most, ws_bytes(q, batch));
  }
  q->tune_nparts = saved;
  return most;
}

extern "C" {

int ffst_spectra(int M, int N, int J, ffst_plan** out) { return ffst_spectra_ex(M, N, J, nullptr, out); }

int ffst_spectra_ex(int M, int N, int J, const ffst_options* opt, ffst_plan** out) {
  const Range range("ffst_spectra_ex");
  const AllocScope alloc_scope;
  if (!out) return fail(FFST_EINVAL, "out must be non-NULL");
  *out = nullptr;
  if (M < 4 || N < 4) return fail(FFST_EINVAL, "image sides must be >= 4 (got %d x %d)", M, N);
  ffst_options o{};
  if (opt) o = *opt;
  if (o.max_scale_min != 0 && o.max_scale_min != 1) return fail(FFST_EINVAL, "max_scale_min must be 0 or 1");
  if (o.shearlet != FFST_SHEARLET_MEYER && o.shearlet != FFST_SHEARLET_MEYER_SMOOTH)
    return fail(FFST_EINVAL, "unknown shearlet %d", o.shearlet);
  if (o.complex_shearlets != 0 && o.complex_shearlets != 1)
    return fail(FFST_EINVAL, "complex_shearlets must be 0 or 1");
  if (o.aux_order < -1 || o.aux_order > 10)
    return fail(FFST_EINVAL, "aux_order must be -1 (C-infinity), 0 (default) or 1 .. 10 (got %d)", o.aux_order);
  if (J <= 0) J = default_scales(M, N);
  if (J < 1 || J > 10) return fail(FFST_EINVAL, "number of scales must be in [1, 10] (got %d)", J);
  if (!supported_length(M) || !supported_length(N) || !supported_row_length(N))
    return fail(FFST_EUNSUPPORTED,
                "GPU path supports sides 2^a 3^b in [4, 4096] (got %d x %d)", M, N);

  ffst_plan* p = new (std::nothrow) ffst_plan();
  if (!p) return fail(FFST_ENOMEM, "host allocation failed");
  p->M = M;
  p->N = N;
  p->J = J;
  p->H = N / 2 + 1;
  // Column lines of the complex buffers are padded by 128 bytes so that the
  // 16-row segments of neighbouring columns do not all share the address
  // bits above 4 KB.
  p->pitch = M >= 64 ? M + 16 : M;
  p->eta = (1 << (J + 2)) - 3;
  p->opt = o;
  p->magic = kMagic;
  if (hipGetDevice(&p->device) != hipSuccess) {
    free_plan(p);
    return fail(FFST_EDEVICE, "hipGetDevice failed");
  }
  // Grid of Sec. 3.5.1: X = 2^(2J-1) ('max') or 2^(2J-2) ('min');
  // Delta = 2X / (L_odd - 1) with L the larger side made odd.
  const int L = std::max(M, N);
  const int L_odd = (L % 2 == 0) ? L + 1 : L;
  const double X = std::ldexp(1.0, 2 * J - 1 - o.max_scale_min);
  p->delta = 2.0 * X / (double)(L_odd - 1);

  std::vector<int> kind, jj, kk;
  index_order(J, kind, jj, kk);
  int *d_kind = nullptr, *d_j = nullptr, *d_k = nullptr;
  int *d_lo = nullptr, *d_hi = nullptr;
  const size_t psi_elems = (size_t)p->eta * M * p->H;
  hipError_t e = dev_alloc(reinterpret_cast<void**>(&p->psi), psi_elems * sizeof(float));
  if (e != hipSuccess) {
    free_plan(p);
    return fail(FFST_ENOMEM, "spectra allocation (%zu bytes): %s", psi_elems * 4, hipGetErrorString(e));
  }
  std::vector<int> lo_init(p->eta, p->H), hi_init(p->eta, -1);
  if ((e = upload(&p->twM, twiddles(M))) != hipSuccess || (e = upload(&p->twN, twiddles(N))) != hipSuccess ||
      (e = upload(&d_kind, kind)) != hipSuccess || (e = upload(&d_j, jj)) != hipSuccess ||
      (e = upload(&d_k, kk)) != hipSuccess || (e = upload(&d_lo, lo_init)) != hipSuccess ||
      (e = upload(&d_hi, hi_init)) != hipSuccess) {
    release(d_kind); release(d_j); release(d_k); release(d_lo); release(d_hi);
    free_plan(p);
    return fail(FFST_ENOMEM, "plan tables: %s", hipGetErrorString(e));
  }
  GenParams g{M, N, p->delta, o.shearlet == FFST_SHEARLET_MEYER_SMOOTH ? 1 : 0, o.aux_order == 0 ? 3 : o.aux_order};
  const bool cplx = o.complex_shearlets == 1;
  e = timed(KID_SPECTRA, nullptr, [&] { return launch_spectra(g, p->eta, d_kind, d_j, d_k, p->psi, nullptr); });
  if (e == hipSuccess && !cplx)
    e = timed(KID_WINDOWS, nullptr, [&] { return launch_windows(p->psi, M, N, p->eta, d_lo, d_hi, nullptr); });
  if (e == hipSuccess) e = hipDeviceSynchronize();
  p->lo.assign(p->eta, 0);
  p->w.assign(p->eta, 0);
  if (e == hipSuccess && cplx) {
    e = one_sided_spectra(p, g, d_kind, d_j, d_k);
  } else if (e == hipSuccess) {
    std::vector<int> hi(p->eta);
    e = hipMemcpy(p->lo.data(), d_lo, p->eta * sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hi.data(), d_hi, p->eta * sizeof(int), hipMemcpyDeviceToHost);
    for (int i = 0; i < p->eta; ++i) {
      if (hi[i] < p->lo[i]) {  // all-zero plane
        p->lo[i] = 0;
        p->w[i] = 0;
      } else {
        p->w[i] = hi[i] - p->lo[i] + 1;
      }
    }
  }
  release(d_kind); release(d_j); release(d_k); release(d_lo); release(d_hi);
  if (e != hipSuccess) {
    free_plan(p);
    return fail(e == hipErrorOutOfMemory ? FFST_ENOMEM : FFST_EDEVICE, "spectra generation: %s",
                hipGetErrorString(e));
  }

  // Compact per-plane windows and the work lists of the column kernels.
  // Real shearlets: half-plane columns [lo, lo + w). Complex shearlets:
  // cyclic full-plane columns (lo + m) mod N, m < w.
  p->off.assign(p->eta, 0);
  long long acc = 0;
  for (int i = 0; i < p->eta; ++i) {
    p->off[i] = acc;
    acc += (long long)p->pitch * p->w[i];
  }
  p->zimg = acc;

  // Plane groups: consecutive spectra whose compact buffer for one image
  // stays within the unit target (one group unless a single image is large).
  const char* env = std::getenv("FFST_CHUNK_MB");
  const long long chunk_mb = env ? std::max(1LL, std::atoll(env)) : 1024LL;
  p->chunk_elems = chunk_mb * (1LL << 20) / (long long)sizeof(float2);
  p->groups = {0};
  long long gsize = 0;
  for (int i = 0; i < p->eta; ++i) {
    const long long sz = (long long)p->pitch * p->w[i];
    if (gsize > 0 && gsize + sz > p->chunk_elems) {
      p->groups.push_back(i);
      gsize = 0;
    }
    gsize += sz;
  }
  p->groups.push_back(p->eta);
  const int ngroups = (int)p->groups.size() - 1;

  // Column passes: half-plane column -> spectra whose window holds it, one
  // CSR per plane group. Complex shearlets: entries (i, 4 m + flags) for the
  // window column m that is c (flag 1) or N - c (flag 2); both flags when
  // c = N - c mod N. In each column the entries with flag 1 or 3 come first
  // (the forward turns its column of the image spectrum into that of N - c
  // once, before the first entry with flag 2).
  std::vector<int> col_ptr, col_planes;
  std::vector<int2> col_ent;
  for (int g = 0; g < ngroups; ++g) {
    col_ptr.push_back(cplx ? (int)col_ent.size() : (int)col_planes.size());
    for (int c = 0; c < p->H; ++c) {
      for (int i = p->groups[g]; i < p->groups[g + 1]; ++i) {
        if (p->w[i] == 0) continue;
        if (!cplx) {
          if (c >= p->lo[i] && c < p->lo[i] + p->w[i]) col_planes.push_back(i);
          continue;
        }
        const int c2 = (p->N - c) % p->N;
        const int m1 = ((c - p->lo[i]) % p->N + p->N) % p->N;
        if (m1 < p->w[i]) col_ent.push_back(make_int2(i, 4 * m1 + (c2 == c ? 3 : 1)));
      }
      if (cplx)
        for (int i = p->groups[g]; i < p->groups[g + 1]; ++i) {
          const int c2 = (p->N - c) % p->N;
          const int m2 = ((c2 - p->lo[i]) % p->N + p->N) % p->N;
          if (p->w[i] > 0 && c2 != c && m2 < p->w[i]) col_ent.push_back(make_int2(i, 4 * m2 + 2));
        }
      col_ptr.push_back(cplx ? (int)col_ent.size() : (int)col_planes.size());
    }
  }
  std::vector<float> psic;
  std::vector<int4> col_hull;
  std::vector<int> acol_ptr;
  std::vector<int2> acol_ent;
  std::vector<int4> acol_hull;
  {
    std::vector<int4> hull_of;
    std::vector<long long> hbase;
    if ((e = spectrum_hulls(p, psic, hull_of, hbase)) != hipSuccess) {
      free_plan(p);
      if (e == hipErrorNotSupported)   // offsets into the hull values are 32-bit
        return fail(FFST_EUNSUPPORTED, "spectrum hulls exceed 2^31 values (%d x %d, J = %d)", M, N, J);
      return fail(e == hipErrorOutOfMemory ? FFST_ENOMEM : FFST_EDEVICE, "spectrum hulls: %s", hipGetErrorString(e));
    }
    if (cplx) {
      for (const int2& en : col_ent) col_hull.push_back(hull_of[hbase[en.x] + (en.y >> 2)]);
      // Adjoint table: the same windows, an entry for column N - c carrying
      // the hull of its line reversed (Psi(-r)); a window column with
      // c = N - c is listed once with each flag.
      const int M = p->M;
      auto reversed = [&](int i, int m) {
        const int4 h = hull_of[hbase[i] + m];
        const int off = (int)psic.size();
        for (int k = 0; k < h.y; ++k) {
          const float v = psic[(size_t)h.z + h.y - 1 - k];
          psic.push_back(v);
        }
        return make_int4(((M - h.x - h.y + 1) % M + M) % M, h.y, off, 0);
      };
      for (int g = 0; g < ngroups; ++g) {
        acol_ptr.push_back((int)acol_ent.size());
        for (int c = 0; c < p->H; ++c) {
          const int c2 = (p->N - c) % p->N;
          for (int i = p->groups[g]; i < p->groups[g + 1]; ++i) {
            if (p->w[i] == 0) continue;
            const int m1 = ((c - p->lo[i]) % p->N + p->N) % p->N;
            const int m2 = ((c2 - p->lo[i]) % p->N + p->N) % p->N;
            if (m1 < p->w[i]) {
              acol_ent.push_back(make_int2(i, 4 * m1 + 1));
              acol_hull.push_back(hull_of[hbase[i] + m1]);
            }
            if (m2 < p->w[i]) {
              acol_ent.push_back(make_int2(i, 4 * m2 + 2));
              acol_hull.push_back(reversed(i, m2));
            }
          }
          acol_ptr.push_back((int)acol_ent.size());
        }
      }
      if (psic.size() > (size_t)INT32_MAX) {
        free_plan(p);
        return fail(FFST_EUNSUPPORTED, "spectrum hulls exceed 2^31 values (%d x %d, J = %d)", M, N, J);
      }
    } else {
      for (int g = 0; g < ngroups; ++g)
        for (int c = 0; c < p->H; ++c)
          for (int t = col_ptr[g * (p->H + 1) + c]; t < col_ptr[g * (p->H + 1) + c + 1]; ++t) {
            const int i = col_planes[t];
            col_hull.push_back(hull_of[hbase[i] + (c - p->lo[i])]);
          }
    }
  }
  std::vector<int> img_lo{0}, img_w{p->H};
  std::vector<long long> img_off{0};
  if ((!p->d_lo && (e = upload(&p->d_lo, p->lo)) != hipSuccess) ||
      (!p->d_w && (e = upload(&p->d_w, p->w)) != hipSuccess) || (e = upload(&p->d_off, p->off)) != hipSuccess || (e = upload(&p->d_img_lo, img_lo)) != hipSuccess ||
      (e = upload(&p->d_img_w, img_w)) != hipSuccess || (e = upload(&p->d_img_off, img_off)) != hipSuccess ||
      (e = upload(&p->d_col_ptr, col_ptr)) != hipSuccess ||
      (e = upload(&p->d_col_planes, col_planes)) != hipSuccess || (e = upload(&p->d_col_ent, col_ent)) != hipSuccess ||
      (e = upload(&p->psic, psic)) != hipSuccess || (e = upload(&p->d_col_hull, col_hull)) != hipSuccess ||
      (e = upload(&p->d_acol_ptr, acol_ptr)) != hipSuccess || (e = upload(&p->d_acol_ent, acol_ent)) != hipSuccess ||
      (e = upload(&p->d_acol_hull, acol_hull)) != hipSuccess) {
    free_plan(p);
    return fail(FFST_ENOMEM, "plan tables: %s", hipGetErrorString(e));
  }
  *out = p;
  if (log_level() >= 1) {
    long long wcols = 0;
    for (int i = 0; i < p->eta; ++i) wcols += p->w[i];
    log_line(1,
         "plan %p: %d x %d, J = %d, eta = %d, %s %s shearlets, aux order %d, %s finest scale; window columns %lld "
         "of %lld, spectrum hull values %zu, plane groups %d; device bytes held by the library %zu",
         (void*)p, M, N, J, p->eta, o.complex_shearlets ? "complex" : "real",
         o.shearlet == FFST_SHEARLET_MEYER_SMOOTH ? "smooth Meyer" : "Meyer", o.aux_order,
         o.max_scale_min ? "'min'" : "'max'", wcols, (long long)p->eta * (o.complex_shearlets ? p->N : p->H),
         psic.size(), ngroups, ffst_device_bytes());
  }
  return ok();
}

int ffst_plan_info(const ffst_plan* p, int* M, int* N, int* J, int* eta) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (M) *M = p->M;
  if (N) *N = p->N;
  if (J) *J = p->J;
  if (eta) *eta = p->eta;
  return ok();
}

size_t ffst_workspace_size(const ffst_plan* p, int batch) {
  if (!plan_ok(p) || batch < 0) return 0;
  return ws_bytes(p, batch);
}

int ffst_get_spectra(const ffst_plan* p, float* dst, int full_plane) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (!dst) return fail(FFST_EINVAL, "dst must be non-NULL");
  if (full_plane != 0 && full_plane != 1) return fail(FFST_EINVAL, "full_plane must be 0 or 1");
  if (p->opt.complex_shearlets) {
    if (!full_plane) return fail(FFST_EINVAL, "one-sided spectra are only available on the full plane");
    hipError_t e = timed(KID_EXPAND, nullptr, [&] {
      return launch_one_sided_expand(p->psip, p->M, p->N, p->eta, p->d_lo, p->d_w, p->d_poff, dst, nullptr);
    });
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return launched(e, "ffst_get_spectra");
  }
  const int cols = full_plane ? p->N : p->H;
  hipError_t e = timed(KID_EXPAND, nullptr, [&] { return launch_expand(p->psi, p->M, p->N, p->eta, cols, dst, nullptr); });
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return launched(e, "ffst_get_spectra");
}

int ffst_plan_windows(const ffst_plan* p, int* first_col, int* last_col) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (!first_col || !last_col) return fail(FFST_EINVAL, "outputs must be non-NULL");
  for (int i = 0; i < p->eta; ++i) {
    first_col[i] = p->w[i] ? p->lo[i] : -1;
    last_col[i] = p->w[i] ? (p->lo[i] + p->w[i] - 1) % (p->opt.complex_shearlets ? p->N : p->H) : -1;
  }
  return ok();
}

static_assert((int)FFST_KIND_LOWPASS == (int)KIND_LOWPASS && (int)FFST_KIND_HORIZONTAL == (int)KIND_H &&
                  (int)FFST_KIND_VERTICAL == (int)KIND_V && (int)FFST_KIND_SEAM == (int)KIND_SEAM,
              "public and internal spectrum kinds must agree");

int ffst_scale_shear(int J, int i, int* kind, int* j, int* k) {
  if (!kind || !j || !k) return fail(FFST_EINVAL, "ffst_scale_shear: outputs must be non-NULL");
  if (J < 1 || J > 10) return fail(FFST_EINVAL, "number of scales must be in [1, 10] (got %d)", J);
  const int eta = (1 << (J + 2)) - 3;
  if (i < 0 || i >= eta) return fail(FFST_EINVAL, "index %d outside [0, %d)", i, eta);
  std::vector<int> kd, jj, kk;
  index_order(J, kd, jj, kk);
  *kind = kd[i];
  *j = kd[i] == KIND_LOWPASS ? -1 : jj[i];
  *k = kk[i];
  return ok();
}

int ffst_shearlet_index(int J, int kind, int j, int k, int* i) {
  if (!i) return fail(FFST_EINVAL, "ffst_shearlet_index: output must be non-NULL");
  if (J < 1 || J > 10) return fail(FFST_EINVAL, "number of scales must be in [1, 10] (got %d)", J);
  std::vector<int> kd, jj, kk;
  index_order(J, kd, jj, kk);
  for (size_t t = 0; t < kd.size(); ++t)
    if (kd[t] == kind && (kind == KIND_LOWPASS || (jj[t] == j && kk[t] == k))) {
      *i = (int)t;
      return ok();
    }
  return fail(FFST_EINVAL, "no plane of kind %d with j = %d, k = %d for J = %d", kind, j, k, J);
}

int ffst_forward(const ffst_plan* p, const float* f, float* coeffs, int batch, void* ws, void* stream) {
  const Range range("ffst_forward");
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (reject_kind(p, false, "ffst_forward") != FFST_OK) return FFST_EINVAL;
  const size_t img = (size_t)p->M * p->N * sizeof(float);
  int st = check_call(p, f, img * (size_t)std::max(batch, 0), coeffs, img * p->eta * (size_t)std::max(batch, 0),
                      batch, ws);
  if (st != FFST_OK || batch == 0) return st;
  const TuningScope tuning(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Schedule sc = schedule(p, batch);
  if (!t_tuning_calls)
    log_line(2, "plan %p ffst_forward: %d image(s), %d per unit, %d line(s) per column", (const void*)p, batch,
         sc.chunk_imgs, sc.fwd_nparts);
  float2* F = static_cast<float2*>(ws);
  float2* Y = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes);
  const long long MH = (long long)p->pitch * p->H;   // one image of F / A
  const long long MN = (long long)p->M * p->N;
  const float scale = (float)(1.0 / ((double)p->M * (double)p->N));

  // row transforms of the images, column-contiguous; the column pass below
  // completes fft2(f) column by column before multiplying by the spectra
  RowArgs ra{const_cast<float*>(f), F, MN, MH, 0, batch, 1, 0, p->M, p->N, p->pitch, image_window(p), p->twN};
  hipError_t e = timed(KID_R2C_IMAGE, s, [&] { return launch_r2c_rows(ra, s); });

  const int ngroups = (int)p->groups.size() - 1;
  for (int img0 = 0; img0 < batch && e == hipSuccess; img0 += sc.chunk_imgs) {
    const int nimg = std::min(sc.chunk_imgs, batch - img0);
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const int p0 = p->groups[g], p1 = p->groups[g + 1];
      const long long base = p->off[p0];
      const long long unit_stride = (p1 < p->eta ? p->off[p1] : p->zimg) - base;
      FwdColArgs fa{p->M, p->N, F + img0 * MH, p->psic, p->d_col_ptr + g * (p->H + 1), p->d_col_planes,
                    p->d_col_hull, nimg, sc.fwd_nparts, p->pitch, plane_windows(p), unit_stride, base, Y, scale,
                    p->twM};
      e = timed(KID_FWD_COLS, s, [&] { return launch_fwd_cols(fa, s); });
      if (e != hipSuccess) break;
      RowArgs rc{coeffs + img0 * p->eta * MN, Y, p->eta * MN, unit_stride, base, nimg, p1 - p0, p0,
                 p->M, p->N, p->pitch, plane_windows(p), p->twN};
      e = timed(KID_C2R_PLANES, s, [&] { return launch_c2r_rows(rc, s); });
    }
  }
  return launched(e, "ffst_forward");
}

int ffst_forward_noalloc(const ffst_plan* p, const float* f, float* coeffs, int batch, void* stream) {
  const Range range("ffst_forward_noalloc");
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (reject_kind(p, false, "ffst_forward_noalloc") != FFST_OK) return FFST_EINVAL;
  if (batch < 0) return fail(FFST_EINVAL, "batch must be >= 0 (got %d)", batch);
  if (batch == 0) return FFST_OK;
  const size_t need = ws_bytes(p, batch);
  if (need > kStaticScratchBytes)
    return fail(FFST_EINVAL,
                "ffst_forward_noalloc: %d image(s) of %d x %d, J = %d need %zu bytes of scratch; the static scratch "
                "holds %zu (use ffst_forward with a workspace, or fewer images per call)",
                batch, p->M, p->N, p->J, need, kStaticScratchBytes);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FFST_EDEVICE, "hipGetDevice failed");
  if (dev != p->device) return fail(FFST_EINVAL, "current device %d is not the plan's device %d", dev, p->device);
  void* ws = nullptr;
  const int st = static_scratch(dev, &ws);
  if (st != FFST_OK) return st;
  const NoTimingScope no_events;   // kernel timing would create HIP events
  return ffst_forward(p, f, coeffs, batch, ws, stream);
}

namespace {

// The real adjoint; with sign_scale (a device scalar s) the coefficients are
// read as s * sign(c).
int adjoint_real(const ffst_plan* p, const float* coeffs, float* f, int batch, void* ws, void* stream,
                 const float* sign_scale, const char* what) {
  const Range range(what);
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (reject_kind(p, false, what) != FFST_OK) return FFST_EINVAL;
  const size_t img = (size_t)p->M * p->N * sizeof(float);
  int st = check_call(p, coeffs, img * p->eta * (size_t)std::max(batch, 0), f, img * (size_t)std::max(batch, 0),
                      batch, ws);
  if (st != FFST_OK || batch == 0) return st;
  const TuningScope tuning(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Schedule sc = schedule(p, batch);
  if (!t_tuning_calls)
    log_line(2, "plan %p %s: %d image(s), %d per unit, %d line(s) per column (%s)", (const void*)p, what, batch,
         sc.chunk_imgs, sc.nparts, sc.fused ? "inverse FFT in the column pass" : "partial sums");
  float2* A = static_cast<float2*>(ws);
  float2* Z = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes);
  float2* P = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes + sc.yz_bytes);
  const long long MH = (long long)p->pitch * p->H;   // one image of F / A
  const long long MN = (long long)p->M * p->N;
  const float scale = (float)(1.0 / ((double)p->M * (double)p->N));
  const int ngroups = (int)p->groups.size() - 1;
  hipError_t e = hipSuccess;
  for (int img0 = 0; img0 < batch && e == hipSuccess; img0 += sc.chunk_imgs) {
    const int nimg = std::min(sc.chunk_imgs, batch - img0);
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const int p0 = p->groups[g], p1 = p->groups[g + 1];
      const long long base = p->off[p0];
      const long long unit_stride = (p1 < p->eta ? p->off[p1] : p->zimg) - base;
      RowArgs rr{const_cast<float*>(coeffs) + img0 * p->eta * MN, Z, p->eta * MN, unit_stride, base, nimg,
                 p1 - p0, p0, p->M, p->N, p->pitch, plane_windows(p), p->twN, sign_scale};
      e = timed(KID_R2C_PLANES, s, [&] { return launch_r2c_rows(rr, s); });
      if (e != hipSuccess) break;
      AdjLineArgs aa{p->M, p->N, Z, unit_stride, base, plane_windows(p), p->psic,
                     p->d_col_ptr + g * (p->H + 1), p->d_col_planes, p->d_col_hull, nimg, sc.nparts, g > 0 ? 1 : 0,
                     sc.fused ? 1 : 0, p->pitch, sc.fused ? A + img0 * MH : P, scale, p->twM};
      e = timed(KID_ADJ_COLS, s, [&] { return launch_adj_lines(aa, s); });
    }
    if (e == hipSuccess && !sc.fused)
      e = timed(KID_IFFT_COLS_IMAGE, s, [&] {
        return launch_line_fft(p->M, A + img0 * MH, nimg * p->H, p->pitch, true, P, sc.nparts,
                               (long long)nimg * MH, p->twM, s);
      });
  }
  if (e == hipSuccess) {
    RowArgs rc{f, A, MN, MH, 0, batch, 1, 0, p->M, p->N, p->pitch, image_window(p), p->twN};
    e = timed(KID_C2R_IMAGE, s, [&] { return launch_c2r_rows(rc, s); });
  }
  return launched(e, what);
}

}  // namespace

int ffst_adjoint(const ffst_plan* p, const float* coeffs, float* f, int batch, void* ws, void* stream) {
  return adjoint_real(p, coeffs, f, batch, ws, stream, nullptr, "ffst_adjoint");
}

int ffst_adjoint_sign(const ffst_plan* p, const float* coeffs, float* f, int batch, const float* scale, void* ws,
                      void* stream) {
  if (!scale) return fail(FFST_EINVAL, "ffst_adjoint_sign: scale must be a non-NULL device pointer");
  return adjoint_real(p, coeffs, f, batch, ws, stream, scale, "ffst_adjoint_sign");
}

int ffst_inverse(const ffst_plan* p, const float* coeffs, float* f, int batch, void* ws, void* stream) {
  return ffst_adjoint(p, coeffs, f, batch, ws, stream);
}

int ffst_forward_complex(const ffst_plan* p, const float* f, float* coeffs, int batch, void* ws, void* stream) {
  const Range range("ffst_forward_complex");
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (reject_kind(p, true, "ffst_forward_complex") != FFST_OK) return FFST_EINVAL;
  const size_t img = (size_t)p->M * p->N * sizeof(float);
  const size_t nb = (size_t)std::max(batch, 0);
  int st = check_call(p, f, img * nb, coeffs, 2 * img * p->eta * nb, batch, ws);
  if (st != FFST_OK || batch == 0) return st;
  const TuningScope tuning(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Schedule sc = schedule(p, batch);
  float2* F = static_cast<float2*>(ws);
  float2* Y = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes);
  float2* C = reinterpret_cast<float2*>(coeffs);
  const long long MH = (long long)p->pitch * p->H;
  const long long MN = (long long)p->M * p->N;
  const float scale = (float)(1.0 / ((double)p->M * (double)p->N));

  // row transforms of the images; the column pass completes fft2(f) per column
  RowArgs ra{const_cast<float*>(f), F, MN, MH, 0, batch, 1, 0, p->M, p->N, p->pitch, image_window(p), p->twN};
  hipError_t e = timed(KID_R2C_IMAGE, s, [&] { return launch_r2c_rows(ra, s); });
  const int ngroups = (int)p->groups.size() - 1;
  for (int img0 = 0; img0 < batch && e == hipSuccess; img0 += sc.chunk_imgs) {
    const int nimg = std::min(sc.chunk_imgs, batch - img0);
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const int p0 = p->groups[g], p1 = p->groups[g + 1];
      const long long base = p->off[p0];
      const long long unit_stride = (p1 < p->eta ? p->off[p1] : p->zimg) - base;
      CFwdColArgs fa{p->M, p->N, F + img0 * MH, p->psic, p->d_col_ptr + g * (p->H + 1), p->d_col_ent,
                     p->d_col_hull, nimg, sc.fwd_nparts, p->pitch, plane_windows(p), unit_stride, base, Y, scale,
                     p->twM};
      e = timed(KID_FWD_COLS_C, s, [&] { return launch_fwd_cols_c(fa, s); });
      if (e != hipSuccess) break;
      CRowArgs rc{C + img0 * p->eta * MN, Y, p->eta * MN, unit_stride, base, nimg, p1 - p0, p0,
                  p->M, p->N, p->pitch, plane_windows(p), p->twN};
      e = timed(KID_C2C_PLANES_INV, s, [&] { return launch_c2c_rows_inv(rc, s); });
    }
  }
  return launched(e, "ffst_forward_complex");
}

int ffst_adjoint_complex(const ffst_plan* p, const float* coeffs, float* f, int batch, void* ws, void* stream) {
  const Range range("ffst_adjoint_complex");
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (reject_kind(p, true, "ffst_adjoint_complex") != FFST_OK) return FFST_EINVAL;
  const size_t img = (size_t)p->M * p->N * sizeof(float);
  const size_t nb = (size_t)std::max(batch, 0);
  int st = check_call(p, coeffs, 2 * img * p->eta * nb, f, img * nb, batch, ws);
  if (st != FFST_OK || batch == 0) return st;
  const TuningScope tuning(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Schedule sc = schedule(p, batch);
  float2* A = static_cast<float2*>(ws);
  float2* Z = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes);
  float2* P = reinterpret_cast<float2*>(static_cast<char*>(ws) + sc.fa_bytes + sc.yz_bytes);
  float2* C = reinterpret_cast<float2*>(const_cast<float*>(coeffs));
  const long long MH = (long long)p->pitch * p->H;
  const long long MN = (long long)p->M * p->N;
  // 1/(M N) of the inverse DFT and 1/2 of the Hermitian part
  const float scale = (float)(0.5 / ((double)p->M * (double)p->N));
  const int ngroups = (int)p->groups.size() - 1;
  hipError_t e = hipSuccess;
  for (int img0 = 0; img0 < batch && e == hipSuccess; img0 += sc.chunk_imgs) {
    const int nimg = std::min(sc.chunk_imgs, batch - img0);
    for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
      const int p0 = p->groups[g], p1 = p->groups[g + 1];
      const long long base = p->off[p0];
      const long long unit_stride = (p1 < p->eta ? p->off[p1] : p->zimg) - base;
      CRowArgs rr{C + img0 * p->eta * MN, Z, p->eta * MN, unit_stride, base, nimg, p1 - p0, p0,
                  p->M, p->N, p->pitch, plane_windows(p), p->twN};
      e = timed(KID_C2C_PLANES_FWD, s, [&] { return launch_c2c_rows_fwd(rr, s); });
      if (e != hipSuccess) break;
      CAdjLineArgs aa{p->M, p->N, Z, unit_stride, base, plane_windows(p), p->psic,
                      p->d_acol_ptr + g * (p->H + 1), p->d_acol_ent, p->d_acol_hull, nimg, sc.nparts, g > 0 ? 1 : 0,
                      sc.fused ? 1 : 0, p->pitch, sc.fused ? A + img0 * MH : P, scale, p->twM};
      e = timed(KID_ADJ_COLS_C, s, [&] { return launch_adj_lines_c(aa, s); });
    }
    if (e == hipSuccess && !sc.fused)
      e = timed(KID_IFFT_COLS_IMAGE, s, [&] {
        return launch_line_fft(p->M, A + img0 * MH, nimg * p->H, p->pitch, true, P, sc.nparts,
                               (long long)nimg * MH, p->twM, s);
      });
  }
  if (e == hipSuccess) {
    RowArgs rc{f, A, MN, MH, 0, batch, 1, 0, p->M, p->N, p->pitch, image_window(p), p->twN};
    e = timed(KID_C2R_IMAGE, s, [&] { return launch_c2r_rows(rc, s); });
  }
  return launched(e, "ffst_adjoint_complex");
}

int ffst_inverse_complex(const ffst_plan* p, const float* coeffs, float* f, int batch, void* ws, void* stream) {
  return ffst_adjoint_complex(p, coeffs, f, batch, ws, stream);
}

int ffst_set_tuning(ffst_plan* p, int nparts, int blocks_per_cu) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  ffst_tuning t{nparts, blocks_per_cu, p->tune_col_values, p->tune_row_block, p->tune_fwd_nparts};
  return ffst_set_tuning_ex(p, &t);
}

int ffst_get_tuning(const ffst_plan* p, int* nparts, int* blocks_per_cu) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (nparts) *nparts = p->tune_nparts;
  if (blocks_per_cu) *blocks_per_cu = p->tune_blocks_per_cu;
  return ok();
}

int ffst_set_tuning_ex(ffst_plan* p, const ffst_tuning* t) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (!t) return fail(FFST_EINVAL, "tuning must be non-NULL");
  if (t->nparts < 0 || t->nparts > 8) return fail(FFST_EINVAL, "nparts must be in [0, 8] (got %d)", t->nparts);
  if (t->fwd_nparts < 0 || t->fwd_nparts > 8)
    return fail(FFST_EINVAL, "fwd_nparts must be in [0, 8] (got %d)", t->fwd_nparts);
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 32)
    return fail(FFST_EINVAL, "blocks_per_cu must be in [0, 32] (got %d)", t->blocks_per_cu);
  const int alt = alt_col_values_of(p);
  if (t->col_values != 0 && !(alt != 0 && t->col_values == alt) && t->col_values != col_values(p->M))
    return fail(FFST_EINVAL, "col_values %d is not compiled for column length %d (default %d, alternative %d)",
                t->col_values, p->M, col_values(p->M), alt);
  if (t->row_block < 0 || t->row_block > 2 || (t->row_block == 2 && !row_block_tunable_of(p)))
    return fail(FFST_EINVAL, "row_block %d is not available for row length %d", t->row_block, p->N);
  p->tune_nparts = t->nparts;
  p->tune_fwd_nparts = t->fwd_nparts;
  p->tune_blocks_per_cu = t->blocks_per_cu;
  p->tune_col_values = t->col_values == col_values(p->M) ? 0 : t->col_values;
  p->tune_row_block = t->row_block == 2 ? 2 : 0;
  log_line(1, "plan %p tuning: nparts %d, fwd_nparts %d, blocks per CU %d, col_values %d, row_block %d", (void*)p,
       t->nparts, t->fwd_nparts, t->blocks_per_cu, t->col_values, t->row_block);
  return ok();
}

int ffst_get_tuning_ex(const ffst_plan* p, ffst_tuning* t) {
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  if (!t) return fail(FFST_EINVAL, "tuning must be non-NULL");
  t->nparts = p->tune_nparts;
  t->fwd_nparts = p->tune_fwd_nparts;
  t->blocks_per_cu = p->tune_blocks_per_cu;
  t->col_values = p->tune_col_values ? p->tune_col_values : col_values(p->M);
  t->row_block = p->tune_row_block == 2 ? 2 : 1;
  return ok();
}

int ffst_tune(ffst_plan* p, const float* f, float* coeffs, float* out, int batch, void* ws, size_t ws_size,
              void* stream, double* best_ms) {
  const Range range("ffst_tune");
  if (!plan_ok(p)) return fail(FFST_EBADPLAN, "invalid plan");
  struct QuietCalls {
    bool saved = t_tuning_calls;
    QuietCalls() { t_tuning_calls = true; }
    ~QuietCalls() { t_tuning_calls = saved; }
  } quiet;
  if (batch < 1) return fail(FFST_EINVAL, "batch must be >= 1 (got %d)", batch);
  if (!f || !coeffs || !out || !ws) return fail(FFST_EINVAL, "buffers must be non-NULL");
  const bool cplx = p->opt.complex_shearlets == 1;
  auto fwd = cplx ? ffst_forward_complex : ffst_forward;
  auto adj = cplx ? ffst_adjoint_complex : ffst_adjoint;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    release_event(a);
    return fail(FFST_EDEVICE, "ffst_tune: hipEventCreate failed");
  }
  const int parts[] = {1, 2, 4, 8};
  const int per_cu[] = {0, 1, 2, 4, 8, 16};
  const int alt = alt_col_values_of(p);
  const int colv[] = {0, alt};
  const int rows[] = {0, 2};
  const int ncolv = alt ? 2 : 1, nrows = row_block_tunable_of(p) ? 2 : 1;
  ffst_tuning saved{};
  saved.nparts = p->tune_nparts;
  saved.fwd_nparts = p->tune_fwd_nparts;
  saved.blocks_per_cu = p->tune_blocks_per_cu;
  saved.col_values = p->tune_col_values;
  saved.row_block = p->tune_row_block;
  auto apply = [p](const ffst_tuning& t) {
    p->tune_nparts = t.nparts;
    p->tune_fwd_nparts = t.fwd_nparts;
    p->tune_blocks_per_cu = t.blocks_per_cu;
    p->tune_col_values = t.col_values;
    p->tune_row_block = t.row_block;
  };
  int st = FFST_OK;
  // best of 3 runs after one warm-up of forward (+ adjoint), in ms
  auto time_it = [&](bool with_adjoint) {
    double t_min = -1.0;
    for (int rep = 0; rep < 4 && st == FFST_OK; ++rep) {
      (void)hipEventRecord(a, s);
      st = fwd(p, f, coeffs, batch, ws, stream);
      if (st == FFST_OK && with_adjoint) st = adj(p, coeffs, out, batch, ws, stream);
      (void)hipEventRecord(b, s);
      float ms = 0.f;
      if (st == FFST_OK && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
        st = fail(FFST_EDEVICE, "ffst_tune: event timing failed");
      if (st == FFST_OK && rep > 0 && (t_min < 0 || ms < t_min)) t_min = ms;
    }
    return t_min;
  };
  // Shapes shared by both directions and the adjoint's split, timed on
  // forward + adjoint with the forward split as it was set; then the
  // forward's own split, timed on the forward alone (it changes nothing else).
  double best = -1.0;
  ffst_tuning best_t = saved;
  for (int iv = 0; iv < ncolv && st == FFST_OK; ++iv)
    for (int ir = 0; ir < nrows && st == FFST_OK; ++ir)
      for (int n : parts) {
        for (int bc : per_cu) {
          const ffst_tuning cand{n, bc, colv[iv], rows[ir], saved.fwd_nparts};
          apply(cand);
          if (ws_bytes(p, batch) > ws_size) continue;
          const double t = time_it(true);
          if (st != FFST_OK) break;
          if (best < 0 || t < best) {
            best = t;
            best_t = cand;
          }
        }
        if (st != FFST_OK) break;
      }
  if (st == FFST_OK && best >= 0) {
    double best_f = -1.0;
    int best_fn = best_t.fwd_nparts;
    for (int fn : parts) {
      ffst_tuning cand = best_t;
      cand.fwd_nparts = fn;
      apply(cand);
      const double t = time_it(false);
      if (st != FFST_OK) break;
      if (best_f < 0 || t < best_f) {
        best_f = t;
        best_fn = fn;
      }
    }
    best_t.fwd_nparts = best_fn;
    apply(best_t);
    if (st == FFST_OK) best = time_it(true);
  }
  release_event(a);
  release_event(b);
  if (st != FFST_OK || best < 0) {
    apply(saved);
    return st != FFST_OK ? st : fail(FFST_EINVAL, "ffst_tune: workspace too small for every candidate");
  }
  apply(best_t);
  if (best_ms) *best_ms = best;
  log_line(1,
       "plan %p tuned for %d image(s): nparts %d, fwd_nparts %d, blocks per CU %d, col_values %d, row_block %d; "
       "forward + adjoint %.4f ms",
       (void*)p, batch, best_t.nparts, best_t.fwd_nparts, best_t.blocks_per_cu,
       best_t.col_values ? best_t.col_values : col_values(p->M), best_t.row_block == 2 ? 2 : 1, best);
  return ok();
}

void ffst_destroy(ffst_plan* p) {
  if (!plan_ok(p)) return;
  log_line(1, "plan %p destroyed", (void*)p);
  (void)hipDeviceSynchronize();
  free_plan(p);
}

const char* ffst_last_error(void) { return g_err.c_str(); }

#ifndef FFST_BUILD_ID
#define FFST_BUILD_ID "unknown"
#endif
const char* ffst_build_id(void) { return FFST_BUILD_ID; }

size_t ffst_device_bytes(void) { return g_live_bytes.load(); }

int ffst_profile_enable(unsigned mask) {
  g_mask.store(mask, std::memory_order_relaxed);
  return FFST_OK;
}

int ffst_profile_read(int id, double* total_ms, long long* launches) {
  if (id < 0 || id >= KID_COUNT) return fail(FFST_EINVAL, "kernel id %d out of range", id);
  drain_profile();
  if (total_ms) *total_ms = g_total_ms[id];
  if (launches) *launches = g_count[id];
  return FFST_OK;
}

int ffst_profile_reset(void) {
  drain_profile();
  std::fill(g_total_ms, g_total_ms + KID_COUNT, 0.0);
  std::fill(g_count, g_count + KID_COUNT, 0LL);
  return FFST_OK;
}

int ffst_num_kernels(void) { return KID_COUNT; }

const char* ffst_kernel_name(int id) { return (id >= 0 && id < KID_COUNT) ? kKernelNames[id] : ""; }

}  // extern "C"
