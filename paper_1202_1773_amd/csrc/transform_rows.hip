// transform_rows.hip -- the FFST hot path on gfx950: layouts, the order of
// the passes, and the row-direction kernels (the column-direction kernels
// are in transform_cols.hip).
//
// Layouts. Every half-plane spectrum (columns c = 0 .. N/2 of a DFT) is kept
// column-contiguous, [c][r]: the image spectrum F, the adjoint's sum A, the
// spectra Psi_i, and the per-spectrum intermediates Y_i / Z_i, which only
// hold the columns [lo_i, lo_i + w_i) where Psi_i is nonzero. The column
// passes read each line of Psi_i only over its shortest cyclic range of
// nonzero rows (the hull), stored compactly at plan creation. The column-
// direction FFTs then stream contiguous lines, and the row kernels move
// between the two layouts through LDS, writing and reading 16 consecutive
// rows of a column at a time (128-byte segments).
//
// Forward (eq. shearletTransform): k_r2c_rows turns the image rows into F
// (real-to-complex along rows, transposed store); k_fwd_cols takes one
// column of F per unit, completes its 2-D FFT with the column FFT in
// registers, and for every spectrum whose window holds the column multiplies
// by that line of Psi_i / (M N), runs the inverse FFT along the column and
// stores the line of Y_i; k_c2r_rows reads Y_i back by row blocks and
// finishes every row with a complex-to-real inverse FFT, writing the
// coefficients. Neither fft2(f) nor Psi_i * F is stored.
//
// Adjoint / inverse (eq. inverseShearletTransform): k_r2c_rows on the
// coefficient rows, storing only the window columns (Z_i); k_adj_lines runs,
// per column line, the forward FFT of every Z_i that has the column,
// multiplies by Psi_i and accumulates the sum over (j, k) in registers, then
// applies the inverse column FFT to the sum (or, when the spectra are split
// over several lines for parallelism, stores partial sums that k_line_fft
// adds in a fixed order before its inverse FFT); k_c2r_rows returns to the
// image.
//
// Real FFT of length N = 2L along a row: z[n] = x[2n] + i x[2n+1],
// Z = FFT_L(z), X[k] = ((Z[k] + conj Z[L-k]) - i W_N^k (Z[k] - conj Z[L-k])) / 2
// for k = 0 .. L. Its inverse forms Z'[k] = (X[k] + conj X[L-k]) +
// i W_N^-k (X[k] - conj X[L-k]), applies the unnormalised inverse FFT_L and
// reads x[2n] = Re, x[2n+1] = Im; that is the unnormalised length-N inverse
// DFT of the Hermitian row.
#include "fft_core.hpp"
#include "internal.hpp"
#include "launch_cfg.hpp"

namespace ffst {
namespace {

// ---------------------------------------------------------------- rows

struct RowJob {
  float* x;                 // real rows: row (img, plane, r) at x + img*x_img_stride + (plane*M + r)*N
  float2* z;                // compact columns: (img, plane, c, r) at z + img*z_img_stride +
                            //   (win.off[plane] - z_off_base) + (c - lo)*zp + r
  long long x_img_stride, z_img_stride, z_off_base;
  int nimg, nplanes, plane0, M, rb;   // rb = rows per block (divides M)
  int zp;                   // complex elements between consecutive columns of z (>= M)
  int stream;               // k_r2c_rows: read x with non-temporal loads
  float inv_nplanes;
  Windows win;
  const float2* twN;        // exp(-2 pi i m / N), m < N
  const float* sign_scale;  // k_r2c_rows_sign: device scalar s; row value x read as s * sign(x)
};

// s * sign(x), sign(0) = 0
__device__ __forceinline__ float sign_times(float x, float s) { return x > 0.f ? s : (x < 0.f ? -s : 0.f); }
__device__ __forceinline__ float2 sign_times(float2 v, float s) {
  return make_float2(sign_times(v.x, s), sign_times(v.y, s));
}

// SMALL: images with fewer than RB rows; the block then covers job.rb rows.
//
// Both row kernels are software-pipelined over the units a block visits: the
// global loads of the next unit are issued before the current unit's FFT, so
// their latency overlaps the arithmetic.
//
// SIGN (k_r2c_rows_sign): the rows are read as s * sign(x), the subgradient of
// s * ||x||_1, so that the adjoint of an l1 term needs no extra pass.
template <int L, int RBM, bool SMALL, bool SIGN>
__device__ __forceinline__ void r2c_rows_body(const RowJob& job) {
  using C = RowCfg<L, RBM>;
  constexpr int V = C::V, G = C::G, N = 2 * L, NT = C::THREADS;
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = group_index<C>();          // row slot (FFT phase)
  const int j = group_lane<C>();
  const int rb = SMALL ? job.rb : C::RB;
  const int tr = threadIdx.x % rb;        // row (transpose phase)
  // first column (transpose phase); with a runtime rb that does not divide
  // NT, threads beyond rb * (NT / rb) sit out (with rb = RB every thread
  // takes part, and the bound stays a compile-time fact)
  const int tc = (!SMALL || threadIdx.x < rb * (NT / rb)) ? threadIdx.x / rb : (1 << 29);
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  TwiddleSeeds<L, V> tw;
  tw.load(j, job.twN, 2);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;
  float sgs = 0.f;
  if constexpr (SIGN) sgs = *job.sign_scale;

  auto load_rows = [&](int u, float2 (&dst)[V]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const float2* xr = reinterpret_cast<const float2*>(job.x + ru.img * job.x_img_stride +
                                                       ((long long)ru.plane * job.M + ru.r0 + (row_ok ? g : 0)) * N);
    if (job.stream) {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = row_ok ? load_stream(xr + j + G * s) : make_float2(0.f, 0.f);
    } else {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = row_ok ? xr[j + G * s] : make_float2(0.f, 0.f);
    }
    if constexpr (SIGN) {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = sign_times(dst[s], sgs);
    }
  };

  float2 nxt[V];
  int u = blockIdx.x;
  if (u < nunits) load_rows(u, nxt);
  for (; u < nunits; u += gridDim.x) {
    float2 v[V];
#pragma unroll
    for (int s = 0; s < V; ++s) v[s] = nxt[s];
    if (u + (int)gridDim.x < nunits) load_rows(u + gridDim.x, nxt);
    fft_group<L, V, false, C::SYNC>(v, j, my, tw);
#pragma unroll
    for (int s = 0; s < V; ++s) my[lpad<V>(j + G * s)] = v[s];
    __syncthreads();

    // X[c] = ((Z[c] + conj Z[L-c]) - i W_N^c (Z[c] - conj Z[L-c])) / 2 for the
    // window columns, stored column-contiguous (rb consecutive rows per column).
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    float2* out = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
    const float2* zr = lds + tr * C::STRIDE;
#pragma unroll 4
    for (int c = lo + tc; c < lo + w; c += cstep) {
      const float2 zc = zr[lpad<V>(c == L ? 0 : c)];
      const float2 zm = conjf2(zr[lpad<V>(c == 0 ? 0 : L - c)]);
      const float2 a = cadd(zc, zm);
      const float2 b = cmul(job.twN[c], csub(zc, zm));
      out[(long long)(c - lo) * job.zp] = make_float2(0.5f * (a.x + b.y), 0.5f * (a.y - b.x));
    }
    __syncthreads();
  }
}

template <int L, int RBM, bool SMALL>
__global__ void __launch_bounds__((RowCfg<L, RBM>::THREADS)) k_r2c_rows(RowJob job) {
  r2c_rows_body<L, RBM, SMALL, false>(job);
}

template <int L, int RBM, bool SMALL>
__global__ void __launch_bounds__((RowCfg<L, RBM>::THREADS)) k_r2c_rows_sign(RowJob job) {
  r2c_rows_body<L, RBM, SMALL, true>(job);
}

template <int L, int RBM, bool SMALL>
__global__ void __launch_bounds__((RowCfg<L, RBM>::THREADS)) k_c2r_rows(RowJob job) {
  using C = RowCfg<L, RBM>;
  constexpr int V = C::V, G = C::G, N = 2 * L, NT = C::THREADS;
  // values each thread moves in the transposed load: k = tc + STEP m, k <= L
  constexpr int STEP = NT / C::RB;
  constexpr int NLD = L / STEP + 1;
  __shared__ float2 lds[C::RB * C::STRIDE];
  __shared__ float2 wsh[L];               // W_N^k, k < L
  const int g = group_index<C>();
  const int j = group_lane<C>();
  const int rb = SMALL ? job.rb : C::RB;
  const int tr = threadIdx.x % rb;
  const int tc = (!SMALL || threadIdx.x < rb * (NT / rb)) ? threadIdx.x / rb : (1 << 29);
  float2* my = lds + g * C::STRIDE;
  TwiddleSeeds<L, V> tw;
  tw.load(j, job.twN, 2);
  for (int k = threadIdx.x; k < L; k += NT) wsh[k] = job.twN[k];
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;
  float2* zr = lds + tr * C::STRIDE;

  // raw half-plane rows X[0 .. L] of a unit (zero outside the window), in
  // the transposed mapping: thread (tr, tc) holds rows tr, columns tc + STEP m
  auto load_cols = [&](int u, float2 (&dst)[NLD]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    const float2* in = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
    const int step = SMALL ? NT / rb : STEP;
#pragma unroll
    for (int m = 0; m < NLD; ++m) {
      const int k = tc + step * m;
      dst[m] = (k <= L && (unsigned)(k - lo) < (unsigned)w) ? in[(long long)(k - lo) * job.zp] : make_float2(0.f, 0.f);
    }
  };

  if constexpr (SMALL) {
    // few rows: no pipelining, every thread may own more columns
    for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
      const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
      const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
      const float2* in = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
      for (int k = tc; k <= L; k += NT / rb)
        zr[lpad<V>(k)] = (unsigned)(k - lo) < (unsigned)w ? in[(long long)(k - lo) * job.zp] : make_float2(0.f, 0.f);
      __syncthreads();
      float2 v[V];
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int k = j + G * s;
        const float2 xk = my[lpad<V>(k)], xm = my[lpad<V>(L - k)];
        const float2 a = make_float2(xk.x + xm.x, xk.y - xm.y);
        const float2 d = make_float2(xk.x - xm.x, xk.y + xm.y);
        const float2 b = cmulc(d, wsh[k]);
        v[s] = make_float2(a.x - b.y, a.y + b.x);
      }
      lds_sync<C::SYNC>();
      fft_group<L, V, true, C::SYNC>(v, j, my, tw);
      if (g < rb) {
        float2* yr = reinterpret_cast<float2*>(job.x + ru.img * job.x_img_stride +
                                               ((long long)ru.plane * job.M + ru.r0 + g) * N);
#pragma unroll
        for (int s = 0; s < V; ++s) yr[j + G * s] = v[s];
      }
      __syncthreads();
    }
  } else {
    float2 nxt[NLD];
    int u = blockIdx.x;
    if (u < nunits) load_cols(u, nxt);
    for (; u < nunits; u += gridDim.x) {
#pragma unroll
      for (int m = 0; m < NLD; ++m) {
        const int k = tc + STEP * m;
        if (k <= L) zr[lpad<V>(k)] = nxt[m];
      }
      __syncthreads();
      if (u + (int)gridDim.x < nunits) load_cols(u + gridDim.x, nxt);
      // Z'[k] = (X[k] + conj X[L-k]) + i conj(W_N^k) (X[k] - conj X[L-k])
      float2 v[V];
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int k = j + G * s;
        const float2 xk = my[lpad<V>(k)], xm = my[lpad<V>(L - k)];
        const float2 a = make_float2(xk.x + xm.x, xk.y - xm.y);
        const float2 d = make_float2(xk.x - xm.x, xk.y + xm.y);
        const float2 b = cmulc(d, wsh[k]);
        v[s] = make_float2(a.x - b.y, a.y + b.x);
      }
      lds_sync<C::SYNC>();
      fft_group<L, V, true, C::SYNC>(v, j, my, tw);
      const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
      float2* yr = reinterpret_cast<float2*>(job.x + ru.img * job.x_img_stride +
                                             ((long long)ru.plane * job.M + ru.r0 + g) * N);
#pragma unroll
      for (int s = 0; s < V; ++s) yr[j + G * s] = v[s];
      __syncthreads();
    }
  }
}

// Odd row lengths N (no half-length packing): a complex FFT of length N per
// row. Forward: x[n] + 0i, X = FFT_N, keep X[c] for the window columns
// (c <= (N-1)/2). Inverse: the window columns give X[c] for c <= (N-1)/2,
// X[N-c] = conj X[c] completes the Hermitian row, and the real part of the
// unnormalised inverse FFT_N is the row (the same scaling as k_c2r_rows).
template <int N, bool SIGN>
__device__ __forceinline__ void r2c_rows_odd_body(const RowJob& job) {
  using C = CRowCfg<N>;
  constexpr int V = C::V, G = C::G, NT = C::THREADS;
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  const int rb = job.rb;
  const int tr = threadIdx.x % rb;
  // threads beyond rb * (NT / rb) sit out of the transposed store
  const int tc = threadIdx.x < rb * (NT / rb) ? threadIdx.x / rb : (1 << 29);
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  const float2* zr = lds + tr * C::STRIDE;
  TwiddleSeeds<N, V> tw;
  tw.load(j, job.twN, 1);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;
  float sgs = 0.f;
  if constexpr (SIGN) sgs = *job.sign_scale;

  auto load_rows = [&](int u, float2 (&dst)[V]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const float* xr = job.x + ru.img * job.x_img_stride + ((long long)ru.plane * job.M + ru.r0 + (row_ok ? g : 0)) * N;
    if (job.stream) {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = make_float2(row_ok ? load_stream(xr + j + G * s) : 0.f, 0.f);
    } else {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = make_float2(row_ok ? xr[j + G * s] : 0.f, 0.f);
    }
    if constexpr (SIGN) {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s].x = sign_times(dst[s].x, sgs);
    }
  };

  float2 nxt[V];
  int u = blockIdx.x;
  if (u < nunits) load_rows(u, nxt);
  for (; u < nunits; u += gridDim.x) {
    float2 v[V];
#pragma unroll
    for (int s = 0; s < V; ++s) v[s] = nxt[s];
    if (u + (int)gridDim.x < nunits) load_rows(u + gridDim.x, nxt);
    fft_group<N, V, false, C::SYNC>(v, j, my, tw);
#pragma unroll
    for (int s = 0; s < V; ++s) my[lpad<V>(j + G * s)] = v[s];
    __syncthreads();
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    float2* out = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
#pragma unroll 4
    for (int m = tc; m < w; m += cstep) out[(long long)m * job.zp] = zr[lpad<V>(lo + m)];
    __syncthreads();
  }
}

template <int N>
__global__ void __launch_bounds__(CRowCfg<N>::THREADS) k_r2c_rows_odd(RowJob job) {
  r2c_rows_odd_body<N, false>(job);
}

template <int N>
__global__ void __launch_bounds__(CRowCfg<N>::THREADS) k_r2c_rows_odd_sign(RowJob job) {
  r2c_rows_odd_body<N, true>(job);
}

template <int N>
__global__ void __launch_bounds__(CRowCfg<N>::THREADS) k_c2r_rows_odd(RowJob job) {
  using C = CRowCfg<N>;
  constexpr int V = C::V, G = C::G, NT = C::THREADS;
  constexpr int H = N / 2 + 1;                       // stored columns 0 .. (N-1)/2
  constexpr int NH = (H + C::GS - 1) / C::GS;        // loads per thread (cstep >= GS)
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  const int rb = job.rb;
  const int tr = threadIdx.x % rb;
  const int tc = threadIdx.x < rb * (NT / rb) ? threadIdx.x / rb : (1 << 29);
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  float2* zr = lds + tr * C::STRIDE;
  TwiddleSeeds<N, V> tw;
  tw.load(j, job.twN, 1);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;

  // columns k = tc + cstep * m of row tr, k < H (zero outside the window)
  auto load_cols = [&](int u, float2 (&dst)[NH]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    const float2* in = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
#pragma unroll
    for (int m = 0; m < NH; ++m) {
      const int k = tc + cstep * m;
      dst[m] = (k < H && (unsigned)(k - lo) < (unsigned)w) ? in[(long long)(k - lo) * job.zp] : make_float2(0.f, 0.f);
    }
  };

  float2 nxt[NH];
  int u = blockIdx.x;
  if (u < nunits) load_cols(u, nxt);
  for (; u < nunits; u += gridDim.x) {
#pragma unroll
    for (int m = 0; m < NH; ++m) {
      const int k = tc + cstep * m;
      if (k < H) {
        zr[lpad<V>(k)] = nxt[m];
        if (k > 0) zr[lpad<V>(N - k)] = conjf2(nxt[m]);
      }
    }
    __syncthreads();
    if (u + (int)gridDim.x < nunits) load_cols(u + gridDim.x, nxt);
    float2 v[V];
#pragma unroll
    for (int s = 0; s < V; ++s) v[s] = my[lpad<V>(j + G * s)];
    lds_sync<C::SYNC>();
    fft_group<N, V, true, C::SYNC>(v, j, my, tw);
    if (row_ok) {
      const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
      float* yr = job.x + ru.img * job.x_img_stride + ((long long)ru.plane * job.M + ru.r0 + g) * N;
#pragma unroll
      for (int s = 0; s < V; ++s) yr[j + G * s] = v[s].x;
    }
    __syncthreads();
  }
}

// Odd row lengths: the odd 3^b from 9 to 2187.
#define FFST_ODD_ROW_CASES(X) X(9) X(27) X(81) X(243) X(729) X(2187)

// Row kernels take the complex length L = N/2: every 2^a 3^b from 2 to 2048.
#define FFST_ROW_CASES(X) X(2) X(3) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) \
  X(6) X(12) X(24) X(48) X(96) X(192) X(384) X(768) X(1536)                              \
  X(9) X(18) X(36) X(72) X(144) X(288) X(576) X(1152)                                   \
  X(27) X(54) X(108) X(216) X(432) X(864) X(1728) X(81) X(162) X(324) X(648) X(1296) X(243) X(486)    \
  X(972) X(1944) X(729) X(1458)

}  // namespace

bool supported_row_length(int N) {
  if (N % 2) {
    switch (N) {
#define CASE(n) case n: return true;
      FFST_ODD_ROW_CASES(CASE)
#undef CASE
      default: return false;
    }
  }
  switch (N / 2) {
#define CASE(n) case n: return true;
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return false;
  }
}

static RowJob make_row_job(const RowArgs& a, int rb_max) {
  RowJob j;
  j.x = a.x;
  j.z = a.z;
  j.x_img_stride = a.x_img_stride;
  j.z_img_stride = a.z_img_stride;
  j.z_off_base = a.z_off_base;
  j.nimg = a.nimg;
  j.nplanes = a.nplanes;
  j.plane0 = a.plane0;
  j.M = a.M;
  j.rb = rows_per_launch(a.M, rb_max, (long long)a.nimg * a.nplanes);
  j.zp = a.zp;
  j.stream = (long long)a.nimg * a.nplanes * a.M * a.N * (long long)sizeof(float) > kStreamBytes;
  j.inv_nplanes = 1.0f / (float)a.nplanes;
  j.win = a.win;
  j.twN = a.twN;
  j.sign_scale = a.sign_scale;
  return j;
}

static hipError_t launch_rows_odd(const RowArgs& a, bool inverse, hipStream_t s) {
  switch (a.N) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const RowJob job = make_row_job(a, CRowCfg<n>::RB);                                           \
    const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);                       \
    const dim3 grid(grid_for(units, CRowCfg<n>::THREADS)), block(CRowCfg<n>::THREADS);           \
    if (inverse)                                                                                  \
      hipLaunchKernelGGL(k_c2r_rows_odd<n>, grid, block, 0, s, job);                              \
    else if (job.sign_scale)                                                                      \
      hipLaunchKernelGGL(k_r2c_rows_odd_sign<n>, grid, block, 0, s, job);                         \
    else                                                                                          \
      hipLaunchKernelGGL(k_r2c_rows_odd<n>, grid, block, 0, s, job);                              \
    return hipGetLastError();                                                                     \
  }
    FFST_ODD_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

// Launchers with the default row blocks (RBM = 1) or, when the call's tuning
// asks for it and the length is compiled for it, doubled ones.
template <int n, int RBM>
hipError_t r2c_rows_with(const RowArgs& a, hipStream_t s) {
  using C = RowCfg<n, RBM>;
  const RowJob job = make_row_job(a, C::RB);
  const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);
  const dim3 grid(grid_for(units, C::THREADS)), block(C::THREADS);
  if (job.sign_scale && job.rb < C::RB)
    hipLaunchKernelGGL((k_r2c_rows_sign<n, RBM, true>), grid, block, 0, s, job);
  else if (job.sign_scale)
    hipLaunchKernelGGL((k_r2c_rows_sign<n, RBM, false>), grid, block, 0, s, job);
  else if (job.rb < C::RB)
    hipLaunchKernelGGL((k_r2c_rows<n, RBM, true>), grid, block, 0, s, job);
  else
    hipLaunchKernelGGL((k_r2c_rows<n, RBM, false>), grid, block, 0, s, job);
  return hipGetLastError();
}

template <int n, int RBM>
hipError_t c2r_rows_with(const RowArgs& a, hipStream_t s) {
  using C = RowCfg<n, RBM>;
  const RowJob job = make_row_job(a, C::RB);
  const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);
  const dim3 grid(grid_for(units, C::THREADS)), block(C::THREADS);
  if (job.rb < C::RB)
    hipLaunchKernelGGL((k_c2r_rows<n, RBM, true>), grid, block, 0, s, job);
  else
    hipLaunchKernelGGL((k_c2r_rows<n, RBM, false>), grid, block, 0, s, job);
  return hipGetLastError();
}

hipError_t launch_r2c_rows(const RowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  if (a.N % 2) return launch_rows_odd(a, false, s);
  switch (a.N / 2) {
#define CASE(n)                                                                    \
  case n:                                                                          \
    if constexpr (row_block_tunable(n))                                            \
      if (t_row_block == 2) return r2c_rows_with<n, 2>(a, s);                      \
    return r2c_rows_with<n, 1>(a, s);
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r_rows(const RowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  if (a.N % 2) return launch_rows_odd(a, true, s);
  switch (a.N / 2) {
#define CASE(n)                                                                    \
  case n:                                                                          \
    if constexpr (row_block_tunable(n))                                            \
      if (t_row_block == 2) return c2r_rows_with<n, 2>(a, s);                      \
    return c2r_rows_with<n, 1>(a, s);
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffst
