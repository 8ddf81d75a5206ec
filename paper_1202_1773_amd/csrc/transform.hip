// transform.hip -- the FFST hot path on gfx950.
//
// Layouts. Every half-plane spectrum (columns c = 0 .. N/2 of a DFT) is kept
// column-contiguous, [c][r]: the image spectrum F, the adjoint's sum A, the
// spectra Psi_i, and the per-spectrum intermediates Y_i / Z_i, which only
// hold the columns [lo_i, lo_i + w_i) where Psi_i is nonzero. The column-
// direction FFTs then stream contiguous lines, and the row kernels move
// between the two layouts through LDS, writing and reading 16 consecutive
// rows of a column at a time (128-byte segments).
//
// Forward (eq. shearletTransform): k_r2c_rows turns the image rows into F
// (real-to-complex along rows, transposed store); k_line_fft transforms F
// along the columns; k_fwd_lines multiplies each column line of F by the
// matching line of Psi_i / (M N), runs the inverse FFT along the column and
// stores Y_i; k_c2r_rows reads Y_i back by row blocks and finishes every row
// with a complex-to-real inverse FFT, writing the coefficients. Psi_i * F is
// never stored.
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
  float inv_nplanes;
  Windows win;
  const float2* twN;        // exp(-2 pi i m / N), m < N
};

// SMALL: images with fewer than RB rows; the block then covers job.rb rows.
//
// Both row kernels are software-pipelined over the units a block visits: the
// global loads of the next unit are issued before the current unit's FFT, so
// their latency overlaps the arithmetic.
template <int L, bool SMALL>
__global__ void __launch_bounds__(RowCfg<L>::THREADS) k_r2c_rows(RowJob job) {
  using C = RowCfg<L>;
  constexpr int V = C::V, G = C::G, N = 2 * L, NT = C::THREADS;
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = threadIdx.x / G;          // row slot (FFT phase)
  const int j = threadIdx.x % G;
  const int rb = SMALL ? job.rb : C::RB;
  const int tr = threadIdx.x % rb;        // row (transpose phase)
  const int tc = threadIdx.x / rb;        // first column (transpose phase)
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  TwiddleRegs<L, V> tw;
  tw.load(j, job.twN, 2);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;

  auto load_rows = [&](int u, float2 (&dst)[V]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const float2* xr = reinterpret_cast<const float2*>(job.x + ru.img * job.x_img_stride +
                                                       ((long long)ru.plane * job.M + ru.r0 + (row_ok ? g : 0)) * N);
#pragma unroll
    for (int s = 0; s < V; ++s) dst[s] = row_ok ? xr[j + G * s] : make_float2(0.f, 0.f);
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
      const float2 zc = zr[lpad<V>(c & (L - 1))];
      const float2 zm = conjf2(zr[lpad<V>((L - c) & (L - 1))]);
      const float2 a = cadd(zc, zm);
      const float2 b = cmul(job.twN[c], csub(zc, zm));
      out[(long long)(c - lo) * job.zp] = make_float2(0.5f * (a.x + b.y), 0.5f * (a.y - b.x));
    }
    __syncthreads();
  }
}

template <int L, bool SMALL>
__global__ void __launch_bounds__(RowCfg<L>::THREADS) k_c2r_rows(RowJob job) {
  using C = RowCfg<L>;
  constexpr int V = C::V, G = C::G, N = 2 * L, NT = C::THREADS;
  // values each thread moves in the transposed load: k = tc + STEP m, k <= L
  constexpr int STEP = NT / C::RB;
  constexpr int NLD = L / STEP + 1;
  __shared__ float2 lds[C::RB * C::STRIDE];
  __shared__ float2 wsh[L];               // W_N^k, k < L
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  const int rb = SMALL ? job.rb : C::RB;
  const int tr = threadIdx.x % rb;
  const int tc = threadIdx.x / rb;
  float2* my = lds + g * C::STRIDE;
  TwiddleRegs<L, V> tw;
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

// ------------------------------------------------------------- columns

// In-place FFT of nlines contiguous lines of length M. Inverse with nparts > 0:
// each line is first replaced by the sum of the same line of `nparts`
// partial arrays (parts + p * part_stride), added in order p = 0, 1, ...
template <int M, bool INV>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) k_line_fft(float2* __restrict__ F, int nlines, int pitch,
                                                                  const float2* __restrict__ parts, int nparts,
                                                                  long long part_stride,
                                                                  const float2* __restrict__ twM) {
  using C = LineCfg<M>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  TwiddleRegs<M, V> tw;
  tw.load(j, twM, 1);
  for (int u = blockIdx.x; u * C::LPB < nlines; u += gridDim.x) {
    const int line = u * C::LPB + g;
    const bool ok = line < nlines;
    float2* base = F + (long long)(ok ? line : 0) * pitch;
    float2 v[V];
    if (nparts > 0) {
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = make_float2(0.f, 0.f);
      // up to 8 partial arrays, all loads issued before the (fixed-order) sums
      constexpr int MAXP = 8;
      float2 t[MAXP][V];
#pragma unroll
      for (int p = 0; p < MAXP; ++p) {
        const float2* pb = parts + p * part_stride + (long long)(ok ? line : 0) * pitch;
#pragma unroll
        for (int s = 0; s < V; ++s) t[p][s] = p < nparts ? pb[j + G * s] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int p = 0; p < MAXP; ++p)
#pragma unroll
        for (int s = 0; s < V; ++s) v[s] = cadd(v[s], t[p][s]);
    } else {
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = base[j + G * s];
    }
    fft_group<M, V, INV, C::SYNC>(v, j, lds + g * C::STRIDE, tw);
    if (ok) {
#pragma unroll
      for (int s = 0; s < V; ++s) base[j + G * s] = v[s];
    }
  }
}

struct FwdLineJob {
  const float2* F;          // [nimg][H][M]
  const float* psi;         // [eta][H][M]
  const int2* lines;        // (spectrum, column) of the unit's lines
  int nlines, nimg, H;
  int pitch;                // complex elements between column lines of F and Y
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};

// Y_i[c - lo_i] = ifft_col(Psi_i[c] * scale * F[c]) for every (line, image).
template <int M>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) k_fwd_lines(FwdLineJob job) {
  using C = LineCfg<M>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  TwiddleRegs<M, V> tw;
  tw.load(j, job.twM, 1);
  const int total = job.nlines * job.nimg;
  // software pipeline: the next unit's F and Psi lines are loaded while the
  // current line is transformed
  float2 fn[V];
  float pn[V];
  auto load_unit = [&](int u) {
    const int q = u * C::LPB + g;
    const int qq = q < total ? q : 0;
    const int img = qq / job.nlines;
    const int2 ln = job.lines[qq % job.nlines];
    const float2* fb = job.F + ((long long)img * job.H + ln.y) * job.pitch;
    const float* pb = job.psi + ((long long)ln.x * job.H + ln.y) * M;
#pragma unroll
    for (int s = 0; s < V; ++s) {
      fn[s] = fb[j + G * s];
      pn[s] = pb[j + G * s];
    }
  };
  int u = blockIdx.x;
  if (u * C::LPB < total) load_unit(u);
  for (; u * C::LPB < total; u += gridDim.x) {
    const int q = u * C::LPB + g;
    const bool ok = q < total;
    const int qq = ok ? q : 0;
    const int img = qq / job.nlines;          // lines of one image are ordered by column,
    const int2 ln = job.lines[qq % job.nlines];  // so neighbouring lines share F[c]
    const int i = ln.x, c = ln.y;
    float2 v[V];
#pragma unroll
    for (int s = 0; s < V; ++s) v[s] = cscale(fn[s], pn[s] * job.scale);
    if ((u + (int)gridDim.x) * C::LPB < total) load_unit(u + gridDim.x);
    fft_group<M, V, true, C::SYNC>(v, j, lds + g * C::STRIDE, tw);
    if (ok) {
      float2* yb = job.Y + img * job.y_img_stride + (job.win.off[i] - job.y_off_base) +
                   (long long)(c - job.win.lo[i]) * job.pitch;
#pragma unroll
      for (int s = 0; s < V; ++s) yb[j + G * s] = v[s];
    }
  }
}

struct AdjLineJob {
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psi;
  const int* col_ptr;       // CSR over columns -> spectra of this plane group
  const int* col_planes;
  int H, nimg, nparts;
  int pitch;                // complex elements between column lines of Z, A and the partial sums
  int accumulate;           // add to the existing partial sums
  float2* out;              // FUSED: A [nimg][H][M]; else partial sums [nparts][nimg][H][M]
  float scale;
  const float2* twM;
};

// Line (img, c, part): sum_i Psi_i[c] * fft_col(Z_i[c - lo_i]) over the spectra
// of column c (part p takes every nparts-th of them); FUSED: scale, inverse
// FFT and store A[c].
template <int M, bool FUSED>
__device__ __forceinline__ void adj_lines_body(const AdjLineJob& job) {
  using C = LineCfg<M>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  float2* my = lds + g * C::STRIDE;
  TwiddleRegs<M, V> tw;
  tw.load(j, job.twM, 1);
  const int total = job.H * job.nimg * job.nparts;
  for (int u = blockIdx.x; u * C::LPB < total; u += gridDim.x) {
    const int q = u * C::LPB + g;
    const bool ok = q < total;
    const int qq = ok ? q : 0;
    const int part = qq % job.nparts;
    const int rest = qq / job.nparts;
    const int img = rest % job.nimg;
    const int c = rest / job.nimg;
    float2 acc[V];
#pragma unroll
    for (int s = 0; s < V; ++s) acc[s] = make_float2(0.f, 0.f);
    const float2* zimg = job.Z + img * job.z_img_stride - job.z_off_base;
    const int q1 = ok ? job.col_ptr[c + 1] : 0;
    int t = job.col_ptr[c] + part;
    // software pipeline: the next spectrum's lines are in flight while the
    // current one is transformed
    float2 zn[V];
    float pn[V];
    if (t < q1) {
      const int i = job.col_planes[t];
      const float2* zb = zimg + job.win.off[i] + (long long)(c - job.win.lo[i]) * job.pitch;
      const float* pb = job.psi + ((long long)i * job.H + c) * M;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        zn[s] = zb[j + G * s];
        pn[s] = pb[j + G * s];
      }
    }
    for (; t < q1; t += job.nparts) {
      float2 v[V];
      float ps[V];
#pragma unroll
      for (int s = 0; s < V; ++s) {
        v[s] = zn[s];
        ps[s] = pn[s];
      }
      const int tn = t + job.nparts;
      if (tn < q1) {
        const int i = job.col_planes[tn];
        const float2* zb = zimg + job.win.off[i] + (long long)(c - job.win.lo[i]) * job.pitch;
        const float* pb = job.psi + ((long long)i * job.H + c) * M;
#pragma unroll
        for (int s = 0; s < V; ++s) {
          zn[s] = zb[j + G * s];
          pn[s] = pb[j + G * s];
        }
      }
      fft_group<M, V, false, C::SYNC>(v, j, my, tw);
#pragma unroll
      for (int s = 0; s < V; ++s) {
        acc[s].x += ps[s] * v[s].x;
        acc[s].y += ps[s] * v[s].y;
      }
    }
#pragma unroll
    for (int s = 0; s < V; ++s) acc[s] = cscale(acc[s], job.scale);
    if constexpr (FUSED) {
      fft_group<M, V, true, C::SYNC>(acc, j, my, tw);
      if (ok) {
        float2* ab = job.out + ((long long)img * job.H + c) * job.pitch;
#pragma unroll
        for (int s = 0; s < V; ++s) ab[j + G * s] = acc[s];
      }
    } else if (ok) {
      float2* pb = job.out + (((long long)part * job.nimg + img) * job.H + c) * job.pitch;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        float2 val = acc[s];
        if (job.accumulate) val = cadd(val, pb[j + G * s]);
        pb[j + G * s] = val;
      }
    }
  }
}

// Up to M = 1024 the body fits 128 registers (4 waves per SIMD) with a few
// spills; larger lengths keep the compiler's own allocation.
template <int M, bool FUSED>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_adj_lines(AdjLineJob job) {
  adj_lines_body<M, FUSED>(job);
}

template <int M, bool FUSED>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) k_adj_lines_wide(AdjLineJob job) {
  adj_lines_body<M, FUSED>(job);
}

// ------------------------------------------------------------ dispatch

// Row kernels take the complex length L = N/2, line kernels the length M.
#define FFST_ROW_CASES(X) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048)
#define FFST_COL_CASES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

}  // namespace

bool supported_length(int L) {
  switch (L) {
#define CASE(n) case n: return true;
    FFST_COL_CASES(CASE)
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
  j.rb = a.M < rb_max ? a.M : rb_max;
  j.zp = a.zp;
  j.inv_nplanes = 1.0f / (float)a.nplanes;
  j.win = a.win;
  j.twN = a.twN;
  return j;
}

hipError_t launch_r2c_rows(const RowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  switch (a.N / 2) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const RowJob job = make_row_job(a, RowCfg<n>::RB);                                            \
    const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);                       \
    const dim3 grid(grid_for(units, RowCfg<n>::THREADS)), block(RowCfg<n>::THREADS);             \
    if (job.rb < RowCfg<n>::RB)                                                                   \
      hipLaunchKernelGGL((k_r2c_rows<n, true>), grid, block, 0, s, job);                              \
    else                                                                                          \
      hipLaunchKernelGGL((k_r2c_rows<n, false>), grid, block, 0, s, job);                             \
    return hipGetLastError();                                                                     \
  }
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r_rows(const RowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  switch (a.N / 2) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const RowJob job = make_row_job(a, RowCfg<n>::RB);                                            \
    const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);                       \
    const dim3 grid(grid_for(units, RowCfg<n>::THREADS)), block(RowCfg<n>::THREADS);             \
    if (job.rb < RowCfg<n>::RB)                                                                   \
      hipLaunchKernelGGL((k_c2r_rows<n, true>), grid, block, 0, s, job);                              \
    else                                                                                          \
      hipLaunchKernelGGL((k_c2r_rows<n, false>), grid, block, 0, s, job);                             \
    return hipGetLastError();                                                                     \
  }
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_line_fft(int M, float2* F, int nlines, int pitch, bool inverse, const float2* parts, int nparts,
                           long long part_stride, const float2* twM, hipStream_t s) {
  if (nlines == 0) return hipSuccess;
  switch (M) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const long long units = (nlines + LineCfg<n>::LPB - 1) / LineCfg<n>::LPB;                     \
    const dim3 grid(grid_for(units, LineCfg<n>::THREADS)), block(LineCfg<n>::THREADS);            \
    if (inverse)                                                                                  \
      hipLaunchKernelGGL((k_line_fft<n, true>), grid, block, 0, s, F, nlines, pitch, parts, nparts, \
                         part_stride, twM);                                                       \
    else                                                                                          \
      hipLaunchKernelGGL((k_line_fft<n, false>), grid, block, 0, s, F, nlines, pitch, parts, nparts, \
                         part_stride, twM);                                                       \
    return hipGetLastError();                                                                     \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd_lines(const FwdLineArgs& a, hipStream_t s) {
  FwdLineJob job{a.F, a.psi, a.lines, a.nlines, a.nimg, a.N / 2 + 1, a.pitch, a.win, a.y_img_stride,
                 a.y_off_base, a.Y, a.scale, a.twM};
  if (job.nlines == 0 || job.nimg == 0) return hipSuccess;
  const long long total = (long long)job.nlines * job.nimg;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const long long units = (total + LineCfg<n>::LPB - 1) / LineCfg<n>::LPB;                      \
    hipLaunchKernelGGL(k_fwd_lines<n>, dim3(grid_for(units, LineCfg<n>::THREADS)),                \
                       dim3(LineCfg<n>::THREADS), 0, s, job);                                     \
    return hipGetLastError();                                                                     \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_lines(const AdjLineArgs& a, hipStream_t s) {
  AdjLineJob job{a.Z, a.z_img_stride, a.z_off_base, a.win, a.psi, a.col_ptr, a.col_planes, a.N / 2 + 1,
                 a.nimg, a.nparts, a.pitch, a.accumulate, a.out, a.scale, a.twM};
  if (job.nimg == 0) return hipSuccess;
  const long long total = (long long)job.H * job.nimg * job.nparts;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const long long units = (total + LineCfg<n>::LPB - 1) / LineCfg<n>::LPB;                      \
    const dim3 grid(grid_for(units, LineCfg<n>::THREADS)), block(LineCfg<n>::THREADS);            \
    if (n <= 1024 && a.fused)                                                                     \
      hipLaunchKernelGGL((k_adj_lines<n, true>), grid, block, 0, s, job);                         \
    else if (n <= 1024)                                                                           \
      hipLaunchKernelGGL((k_adj_lines<n, false>), grid, block, 0, s, job);                        \
    else if (a.fused)                                                                             \
      hipLaunchKernelGGL((k_adj_lines_wide<n, true>), grid, block, 0, s, job);                    \
    else                                                                                          \
      hipLaunchKernelGGL((k_adj_lines_wide<n, false>), grid, block, 0, s, job);                   \
    return hipGetLastError();                                                                     \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffst
