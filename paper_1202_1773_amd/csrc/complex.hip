// complex.hip -- the FFST with complex shearlets (one-sided spectra, Sec. 3.8.2).
//
// Coefficients: c_i = ifft2(Psi+_i * fft2(f)), complex, for a real image f.
// Psi+_i is not even, so the coefficient rows are complex and the row pass is
// a complex FFT of length N over the full plane. The image spectrum F is
// still kept on the half plane (f is real): full-plane column c > N/2 is
// read as conj F(-r, N - c). Psi+_i is stored compactly over a cyclic range
// of full-plane columns (one lobe, plus the Nyquist values that stay two-
// sided), so the intermediates Y_i / Z_i hold only those columns.
//
// Forward: the real transform's image row pass gives the row transforms of
// f on the half plane; k_fwd_cols_c takes one half-plane column c per unit,
// completes fft2(f) at c with the column FFT in registers, and for every
// window column of a Psi+_i that is c or N - c multiplies by that line of
// Psi+_i / (M N) (read over its hull of nonzero rows) and runs the inverse
// column FFT into Y_i; column N - c is conj X(-r) of column c, formed once
// per unit through LDS. k_c2c_rows_inv runs the inverse row FFT over the
// window columns and writes full complex rows of c_i.
//
// Adjoint (for real images): Re sum_i ifft2(Psi+_i fft2(c_i)). With
// X = sum_i Psi+_i fft2(c_i) this is the inverse DFT of the Hermitian part
// (X(w) + conj X(-w)) / 2, whose half plane the real transform's last passes
// turn into the image. k_c2c_rows_fwd runs the forward row FFT of each
// coefficient row and stores its window columns Z_i; k_adj_lines_c, per
// half-plane column c, transforms along the column every Z_i column that is
// c or N - c, multiplies by Psi+_i (over its hull) and accumulates both sums
// in registers, then forms (X(r, c) + conj X(-r, N - c)) / 2 through LDS.
#include "fft_core.hpp"
#include "internal.hpp"
#include "launch_cfg.hpp"

namespace ffst {
namespace {

struct CRowJob {
  float2* x;                // complex rows: (img, plane, r) at x + img*x_img_stride + (plane*M + r)*L
  float2* z;                // window columns: (img, plane, m, r) at z + img*z_img_stride +
                            //   (win.off[plane] - z_off_base) + m*zp + r
  long long x_img_stride, z_img_stride, z_off_base;
  int nimg, nplanes, plane0, M, rb, zp;
  int stream;               // k_c2c_rows_fwd: read x with non-temporal loads
  float inv_nplanes;
  Windows win;
  const float2* twN;        // exp(-2 pi i m / L), m < L
};

// Inverse row FFT: the window columns of each row become a full complex row.
template <int L>
__global__ void __launch_bounds__(CRowCfg<L>::THREADS) k_c2c_rows_inv(CRowJob job) {
  using C = CRowCfg<L>;
  constexpr int V = C::V, G = C::G, NT = C::THREADS;
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = group_index<C>();          // row slot (FFT phase)
  const int j = group_lane<C>();
  const int rb = job.rb;
  const int tr = threadIdx.x % rb;        // row (transpose phase)
  // first column (transpose phase); threads beyond rb * (NT / rb) sit out
  const int tc = threadIdx.x < rb * (NT / rb) ? threadIdx.x / rb : (1 << 29);
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  float2* zr = lds + tr * C::STRIDE;
  TwiddleSeeds<L, V> tw;
  tw.load(j, job.twN, 1);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;

  // columns k = tc + cstep * m of row tr (zero outside the window); V values
  // cover the row since cstep * V >= L
  auto load_cols = [&](int u, float2 (&dst)[V]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    const float2* in = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
#pragma unroll
    for (int m = 0; m < V; ++m) {
      const int k = tc + cstep * m;
      const int cm = k >= lo ? k - lo : k - lo + L;
      dst[m] = (k < L && cm < w) ? in[(long long)cm * job.zp] : make_float2(0.f, 0.f);
    }
  };

  float2 nxt[V];
  int u = blockIdx.x;
  if (u < nunits) load_cols(u, nxt);
  for (; u < nunits; u += gridDim.x) {
#pragma unroll
    for (int m = 0; m < V; ++m) {
      const int k = tc + cstep * m;
      if (k < L) zr[lpad<V>(k)] = nxt[m];
    }
    __syncthreads();
    if (u + (int)gridDim.x < nunits) load_cols(u + gridDim.x, nxt);
    float2 v[V];
#pragma unroll
    for (int s = 0; s < V; ++s) v[s] = my[lpad<V>(j + G * s)];
    lds_sync<C::SYNC>();
    fft_group<L, V, true, C::SYNC>(v, j, my, tw);
    if (row_ok) {
      const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
      float2* yr = job.x + ru.img * job.x_img_stride + ((long long)ru.plane * job.M + ru.r0 + g) * L;
#pragma unroll
      for (int s = 0; s < V; ++s) yr[j + G * s] = v[s];
    }
    __syncthreads();
  }
}

// Forward row FFT of full complex rows; the window columns are stored
// column-contiguous (rb consecutive rows per column).
template <int L>
__global__ void __launch_bounds__(CRowCfg<L>::THREADS) k_c2c_rows_fwd(CRowJob job) {
  using C = CRowCfg<L>;
  constexpr int V = C::V, G = C::G, NT = C::THREADS;
  __shared__ float2 lds[C::RB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  const int rb = job.rb;
  const int tr = threadIdx.x % rb;
  const int tc = threadIdx.x < rb * (NT / rb) ? threadIdx.x / rb : (1 << 29);
  const int cstep = NT / rb;
  const bool row_ok = g < rb;
  float2* my = lds + g * C::STRIDE;
  const float2* zr = lds + tr * C::STRIDE;
  TwiddleSeeds<L, V> tw;
  tw.load(j, job.twN, 1);
  const int bpp = job.M / rb;
  const int nunits = job.nimg * job.nplanes * bpp;

  auto load_rows = [&](int u, float2 (&dst)[V]) {
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const float2* xr = job.x + ru.img * job.x_img_stride +
                       ((long long)ru.plane * job.M + ru.r0 + (row_ok ? g : 0)) * L;
    if (job.stream) {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = row_ok ? load_stream(xr + j + G * s) : make_float2(0.f, 0.f);
    } else {
#pragma unroll
      for (int s = 0; s < V; ++s) dst[s] = row_ok ? xr[j + G * s] : make_float2(0.f, 0.f);
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
    const RowUnit ru = row_unit(u, bpp, job.nplanes, job.inv_nplanes, rb, job.plane0);
    const int lo = job.win.lo[ru.plane], w = job.win.w[ru.plane];
    float2* out = job.z + ru.img * job.z_img_stride + (job.win.off[ru.plane] - job.z_off_base) + ru.r0 + tr;
#pragma unroll 4
    for (int m = tc; m < w; m += cstep) out[(long long)m * job.zp] = zr[lpad<V>(wrap_once(lo + m, L))];
    __syncthreads();
  }
}

// Index m of element e of a column line inside the line's cyclic hull
// [r_lo, r_lo + K) (mod L), or a value >= K when e lies outside it.
template <int L>
__device__ __forceinline__ int chull_index(int e, int r_lo) {
  const int d = e - r_lo;
  return d < 0 ? d + L : d;
}

struct CFwdColJob {
  const float2* F;
  const float* psic;
  const int* col_ptr;
  const int2* col_ent;
  const int4* col_hull;
  int H, nimg, nparts;
  int pitch;
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};

// Unit (c, img, part): X = fft_col of the row transforms at half-plane
// column c; then, for every nparts-th entry of the column (from the part's
// index), Y_i[m] = ifft_col(Psi+_i[m] * scale * X') with X' = X for flags 1
// and 3 (the window column is c) and X'(r) = conj X(-r) for flag 2 (it is
// N - c). The column's entries with flag 2 come last, so X is turned into
// X' once, at the first of them. Units run column-major (the images of one
// column share its spectrum lines).
template <int M>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) k_fwd_cols_c(CFwdColJob job) {
  using C = LineCfg<M>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  float2* my = lds + g * C::STRIDE;
  TwiddleSeeds<M, V> tw;
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
    const float2* fb = job.F + ((long long)img * job.H + c) * job.pitch;
    float2 x[V];
#pragma unroll
    for (int s = 0; s < V; ++s) x[s] = fb[j + G * s];
    fft_group<M, V, false, C::SYNC>(x, j, my, tw);
    float2* yimg = job.Y + img * job.y_img_stride - job.y_off_base;
    const int q1 = ok ? job.col_ptr[c + 1] : 0;
    int t = job.col_ptr[c] + part;
    bool mirrored = false;
    float pn[V];
    auto load_psi = [&](int tt) {
      const int4 hl = job.col_hull[tt];
      const float* pb = job.psic + hl.z;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int m = chull_index<M>(j + G * s, hl.x);
        pn[s] = m < hl.y ? pb[m] * job.scale : 0.f;
      }
    };
    if (t < q1) load_psi(t);
    for (; t < q1; t += job.nparts) {
      const int2 e = job.col_ent[t];
      if ((e.y & 3) == 2 && !mirrored) {
        // X'(r) = conj X(-r mod M), through the group's LDS
#pragma unroll
        for (int s = 0; s < V; ++s) my[lpad<V>(j + G * s)] = x[s];
        lds_sync<C::SYNC>();
#pragma unroll
        for (int s = 0; s < V; ++s) x[s] = conjf2(my[lpad<V>(mirror_index(j + G * s, M))]);
        lds_sync<C::SYNC>();
        mirrored = true;
      }
      float2 v[V];
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = cscale(x[s], pn[s]);
      if (t + job.nparts < q1) load_psi(t + job.nparts);
      fft_group<M, V, true, C::SYNC>(v, j, my, tw);
      float2* yb = yimg + job.win.off[e.x] + (long long)(e.y >> 2) * job.pitch;
#pragma unroll
      for (int s = 0; s < V; ++s) yb[j + G * s] = v[s];
    }
  }
}

struct CAdjLineJob {
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psic;
  const int* col_ptr;
  const int2* col_ent;
  const int4* col_hull;
  int H, nimg, nparts;
  int pitch;
  int accumulate;
  float2* out;              // FUSED: A [nimg][H][pitch]; else partial sums [nparts][nimg][H][pitch]
  float scale;              // 1 / (2 M N)
  const float2* twM;
};

// Line (img, c, part): A[c](r) = scale * (X1(r) + conj X2(-r)), X1 the sum
// of Psi+_i[m] fft_col(Z_i[m]) over the windows that hold column c, X2 the
// same over those that hold N - c (part p takes every nparts-th entry). The
// second sum is accumulated directly: conj (Psi X)(-r) = Psi(-r)
// fft_col(conj z)(r) for a real Psi and X = fft_col(z), so an entry for
// column N - c (flag 2) transforms the conjugated line and carries the
// spectrum line reversed (Psi(-r), stored so at plan creation). A window
// column with c = N - c enters the adjoint's table twice, once each way.
template <int M, bool FUSED>
__device__ __forceinline__ void adj_lines_c_body(const CAdjLineJob& job) {
  using C = LineCfg<M>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  float2* my = lds + g * C::STRIDE;
  TwiddleSeeds<M, V> tw;
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
    float2 zn[V];
    float pn[V];
    int fn = 0;
    auto load_entry = [&](int tt) {
      const int2 e = job.col_ent[tt];
      const int4 hl = job.col_hull[tt];
      fn = e.y & 3;
      const float2* zb = zimg + job.win.off[e.x] + (long long)(e.y >> 2) * job.pitch;
      const float* pb = job.psic + hl.z;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        zn[s] = zb[j + G * s];
        const int m = chull_index<M>(j + G * s, hl.x);
        pn[s] = m < hl.y ? pb[m] : 0.f;
      }
    };
    if (t < q1) load_entry(t);
    for (; t < q1; t += job.nparts) {
      float2 v[V];
      float ps[V];
      const int fl = fn;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        v[s] = fl == 2 ? conjf2(zn[s]) : zn[s];
        ps[s] = pn[s];
      }
      if (t + job.nparts < q1) load_entry(t + job.nparts);
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

template <int M, bool FUSED>
__global__ void __launch_bounds__(LineCfg<M>::THREADS) k_adj_lines_c(CAdjLineJob job) {
  adj_lines_c_body<M, FUSED>(job);
}

// Complex row kernels take the full length N, line kernels the length M.
// Powers of two, 3 * 2^k and 9 * 2^k.
#define FFST_CROW_CASES(X) X(4) X(6) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) \
  X(12) X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)                             \
  X(9) X(18) X(36) X(72) X(144) X(288) X(576) X(1152) X(2304)                               \
  X(27) X(54) X(108) X(216) X(432) X(864) X(1728) X(3456) X(81) X(162) X(324) X(648) X(1296) X(2592)  \
  X(243) X(486) X(972) X(1944) X(3888) X(729) X(1458) X(2916) X(2187)
#define FFST_CCOL_CASES(X) FFST_CROW_CASES(X)

CRowJob make_crow_job(const CRowArgs& a, int rb_max) {
  CRowJob j;
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
  j.stream = (long long)a.nimg * a.nplanes * a.M * a.N * (long long)sizeof(float2) > kStreamBytes;
  j.zp = a.zp;
  j.inv_nplanes = 1.0f / (float)a.nplanes;
  j.win = a.win;
  j.twN = a.twN;
  return j;
}

}  // namespace

hipError_t launch_c2c_rows_inv(const CRowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  switch (a.N) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const CRowJob job = make_crow_job(a, CRowCfg<n>::RB);                                         \
    const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);                       \
    hipLaunchKernelGGL(k_c2c_rows_inv<n>, dim3(grid_for(units, CRowCfg<n>::THREADS)),             \
                       dim3(CRowCfg<n>::THREADS), 0, s, job);                                     \
    return hipGetLastError();                                                                     \
  }
    FFST_CROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2c_rows_fwd(const CRowArgs& a, hipStream_t s) {
  if (a.nimg == 0 || a.nplanes == 0) return hipSuccess;
  switch (a.N) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const CRowJob job = make_crow_job(a, CRowCfg<n>::RB);                                         \
    const long long units = (long long)a.nimg * a.nplanes * (a.M / job.rb);                       \
    hipLaunchKernelGGL(k_c2c_rows_fwd<n>, dim3(grid_for(units, CRowCfg<n>::THREADS)),             \
                       dim3(CRowCfg<n>::THREADS), 0, s, job);                                     \
    return hipGetLastError();                                                                     \
  }
    FFST_CROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd_cols_c(const CFwdColArgs& a, hipStream_t s) {
  CFwdColJob job{a.F, a.psic, a.col_ptr, a.col_ent, a.col_hull, a.N / 2 + 1, a.nimg, a.nparts, a.pitch, a.win,
                 a.y_img_stride, a.y_off_base, a.Y, a.scale, a.twM};
  if (job.nimg == 0) return hipSuccess;
  if (job.nparts < 1) return hipErrorInvalidValue;
  const long long total = (long long)job.H * job.nimg * job.nparts;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const long long units = (total + LineCfg<n>::LPB - 1) / LineCfg<n>::LPB;                      \
    hipLaunchKernelGGL(k_fwd_cols_c<n>, dim3(grid_for(units, LineCfg<n>::THREADS)),               \
                       dim3(LineCfg<n>::THREADS), 0, s, job);                                     \
    return hipGetLastError();                                                                     \
  }
    FFST_CCOL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_lines_c(const CAdjLineArgs& a, hipStream_t s) {
  CAdjLineJob job{a.Z, a.z_img_stride, a.z_off_base, a.win, a.psic, a.col_ptr, a.col_ent, a.col_hull, a.N / 2 + 1,
                  a.nimg, a.nparts, a.pitch, a.accumulate, a.out, a.scale, a.twM};
  if (job.nimg == 0) return hipSuccess;
  const long long total = (long long)job.H * job.nimg * job.nparts;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n: {                                                                                       \
    const long long units = (total + LineCfg<n>::LPB - 1) / LineCfg<n>::LPB;                      \
    const dim3 grid(grid_for(units, LineCfg<n>::THREADS)), block(LineCfg<n>::THREADS);            \
    if (a.fused)                                                                                  \
      hipLaunchKernelGGL((k_adj_lines_c<n, true>), grid, block, 0, s, job);                       \
    else                                                                                          \
      hipLaunchKernelGGL((k_adj_lines_c<n, false>), grid, block, 0, s, job);                      \
    return hipGetLastError();                                                                     \
  }
    FFST_CCOL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffst
