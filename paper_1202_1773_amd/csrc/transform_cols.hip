// transform_cols.hip -- the column-direction passes of the FFST hot path on
// gfx950: in-place line FFTs of half-plane spectra (k_line_fft), the
// forward column pass (k_fwd_cols: per column, the image's column FFT, then
// the multiply + inverse column FFT for every spectrum that reaches the
// column) and the adjoint's column FFT + multiply + sum over spectra
// (k_adj_lines). The layouts and the order of the passes are described with
// the row kernels.
#include "fft_core.hpp"
#include "internal.hpp"
#include "launch_cfg.hpp"

#include <algorithm>

namespace ffst {
namespace {

// In-place FFT of nlines contiguous lines of length M. PARTS (inverse with
// nparts > 0): each line is first replaced by the sum of the same line of
// `nparts` partial arrays (parts + p * part_stride), added in order
// p = 0, 1, ...; a separate instantiation, so that the plain transform keeps
// its registers.
template <int M, int VV, bool INV, bool PARTS>
__global__ void __launch_bounds__((LineCfg<M, VV>::THREADS)) k_line_fft(float2* __restrict__ F, int nlines, int pitch,
                                                                      const float2* __restrict__ parts, int nparts,
                                                                      long long part_stride,
                                                                      const float2* __restrict__ twM) {
  using C = LineCfg<M, VV>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::LPB * C::STRIDE];
  const int g = group_index<C>();
  const int j = group_lane<C>();
  TwiddleRegs<M, V> tw;
  tw.load(j, twM, 1);
  for (int u = blockIdx.x; u * C::LPB < nlines; u += gridDim.x) {
    const int line = u * C::LPB + g;
    const bool ok = line < nlines;
    float2* base = F + (long long)(ok ? line : 0) * pitch;
    float2 v[V];
    if constexpr (PARTS) {
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = make_float2(0.f, 0.f);
      // the partial arrays in groups of MAXP (64 values per lane in flight for
      // 8-value lanes, fewer for wider lanes),
      // every load of a group issued before its sums; sums in order p = 0, 1, ...
      constexpr int MAXP = V <= 8 ? 8 : 2;
      for (int p0 = 0; p0 < nparts; p0 += MAXP) {
        float2 t[MAXP][V];
#pragma unroll
        for (int k = 0; k < MAXP; ++k) {
          const int pk = p0 + k < nparts ? p0 + k : nparts - 1;   // in bounds even if loaded early
          const float2* pb = parts + pk * part_stride + (long long)(ok ? line : 0) * pitch;
#pragma unroll
          for (int s = 0; s < V; ++s) t[k][s] = p0 + k < nparts ? pb[j + G * s] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < MAXP; ++k)
#pragma unroll
          for (int s = 0; s < V; ++s) v[s] = cadd(v[s], t[k][s]);
      }
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

// Index m of element e of a column line inside the line's cyclic hull
// [r_lo, r_lo + K) (mod L), or a value >= K when e lies outside it.
template <int L>
__device__ __forceinline__ int hull_index(int e, int r_lo) {
  const int d = e - r_lo;
  return d < 0 ? d + L : d;
}

struct FwdColJob {
  const float2* F;          // row transforms of the images, column-contiguous [nimg][H][pitch]
  const float* psic;        // compact spectrum lines (see FwdColArgs)
  const int* col_ptr;       // CSR over columns -> spectra of this plane group
  const int* col_planes;
  const int4* col_hull;     // hull of every CSR entry's line
  int H, nimg, nparts;
  int pitch;                // complex elements between column lines of F and Y
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};

// Unit (c, img, part): the column FFT of the image's row transforms at
// column c gives F[c] (the image spectrum's column, kept in registers);
// then, for every nparts-th spectrum i whose window holds c (starting at
// the part's index),
//   Y_i[c - lo_i] = ifft_col(Psi_i[c] * scale * F[c]),
// with Psi_i[c] read only inside its hull. Several parts per column (small
// batches) repeat the column FFT so that a column's spectra run on several
// lines in parallel. Units run column-major (images of one column next to
// each other share the spectrum lines). The next spectrum's line is loaded
// while the current one is transformed.
template <int M, int VV>
__global__ void __launch_bounds__((LineCfg<M, VV>::THREADS)) k_fwd_cols(FwdColJob job) {
  using C = LineCfg<M, VV>;
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
    float2 f[V];
#pragma unroll
    for (int s = 0; s < V; ++s) f[s] = fb[j + G * s];
    fft_group<M, V, false, C::SYNC>(f, j, my, tw);
    float2* yimg = job.Y + img * job.y_img_stride - job.y_off_base;
    const int q1 = ok ? job.col_ptr[c + 1] : 0;
    int t = job.col_ptr[c] + part;
    float pn[V];
    auto load_psi = [&](int tt) {
      const int4 hl = job.col_hull[tt];
      const float* pb = job.psic + hl.z;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        const int m = hull_index<M>(j + G * s, hl.x);
        pn[s] = m < hl.y ? pb[m] * job.scale : 0.f;
      }
    };
    if (t < q1) load_psi(t);
    for (; t < q1; t += job.nparts) {
      const int i = job.col_planes[t];
      float2 v[V];
#pragma unroll
      for (int s = 0; s < V; ++s) v[s] = cscale(f[s], pn[s]);
      if (t + job.nparts < q1) load_psi(t + job.nparts);
      fft_group<M, V, true, C::SYNC>(v, j, my, tw);
      float2* yb = yimg + job.win.off[i] + (long long)(c - job.win.lo[i]) * job.pitch;
#pragma unroll
      for (int s = 0; s < V; ++s) yb[j + G * s] = v[s];
    }
  }
}

struct AdjLineJob {
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psic;        // compact spectrum lines (see FwdColArgs)
  const int* col_ptr;       // CSR over columns -> spectra of this plane group
  const int* col_planes;
  const int4* col_hull;     // hull of every CSR entry's line
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
template <int M, int VV, bool FUSED>
__device__ __forceinline__ void adj_lines_body(const AdjLineJob& job) {
  using C = LineCfg<M, VV>;
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
    // software pipeline: the next spectrum's lines are in flight while the
    // current one is transformed
    float2 zn[V];
    float pn[V];
    if (t < q1) {
      const int i = job.col_planes[t];
      const int4 hl = job.col_hull[t];
      const float2* zb = zimg + job.win.off[i] + (long long)(c - job.win.lo[i]) * job.pitch;
      const float* pb = job.psic + hl.z;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        zn[s] = zb[j + G * s];
        const int m = hull_index<M>(j + G * s, hl.x);
        pn[s] = m < hl.y ? pb[m] : 0.f;
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
        const int4 hl = job.col_hull[tn];
        const float2* zb = zimg + job.win.off[i] + (long long)(c - job.win.lo[i]) * job.pitch;
        const float* pb = job.psic + hl.z;
#pragma unroll
        for (int s = 0; s < V; ++s) {
          zn[s] = zb[j + G * s];
          const int m = hull_index<M>(j + G * s, hl.x);
          pn[s] = m < hl.y ? pb[m] : 0.f;
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

// The compiler's own register allocation (no occupancy target): capping
// the 512-point body at 128 registers (4 waves per SIMD) spilled to scratch
// and was slower than 3 waves without spills.
template <int M, int VV, bool FUSED>
__global__ void __launch_bounds__((LineCfg<M, VV>::THREADS)) k_adj_lines(AdjLineJob job) {
  adj_lines_body<M, VV, FUSED>(job);
}

// Launches with the default lane width (VV = 0) or, when the call's tuning
// asks for it and it is compiled, the alternative one.
template <int n, int VV>
hipError_t line_fft_with(float2* F, int nlines, int pitch, bool inverse, const float2* parts, int nparts,
                         long long part_stride, const float2* twM, hipStream_t s) {
  using C = LineCfg<n, VV>;
  const long long units = (nlines + C::LPB - 1) / C::LPB;
  const dim3 grid(grid_for(units, C::THREADS)), block(C::THREADS);
  if (inverse && nparts > 0)
    hipLaunchKernelGGL((k_line_fft<n, VV, true, true>), grid, block, 0, s, F, nlines, pitch, parts, nparts,
                       part_stride, twM);
  else if (inverse)
    hipLaunchKernelGGL((k_line_fft<n, VV, true, false>), grid, block, 0, s, F, nlines, pitch, parts, nparts,
                       part_stride, twM);
  else
    hipLaunchKernelGGL((k_line_fft<n, VV, false, false>), grid, block, 0, s, F, nlines, pitch, parts, nparts,
                       part_stride, twM);
  return hipGetLastError();
}

template <int n, int VV>
hipError_t fwd_cols_with(const FwdColJob& job, long long total, hipStream_t s) {
  using C = LineCfg<n, VV>;
  const long long units = (total + C::LPB - 1) / C::LPB;
  hipLaunchKernelGGL((k_fwd_cols<n, VV>), dim3(grid_for(units, C::THREADS)), dim3(C::THREADS), 0, s, job);
  return hipGetLastError();
}

template <int n, int VV>
hipError_t adj_lines_with(const AdjLineJob& job, long long total, bool fused, hipStream_t s) {
  using C = LineCfg<n, VV>;
  const long long units = (total + C::LPB - 1) / C::LPB;
  const dim3 grid(grid_for(units, C::THREADS)), block(C::THREADS);
  if (fused)
    hipLaunchKernelGGL((k_adj_lines<n, VV, true>), grid, block, 0, s, job);
  else
    hipLaunchKernelGGL((k_adj_lines<n, VV, false>), grid, block, 0, s, job);
  return hipGetLastError();
}

// true when this call's tuning asks for the alternative lane width of n
inline bool alt_cols_requested(int n) { return t_col_values != 0 && t_col_values == alt_col_values(n); }

// Line kernels take the length M: every 2^a 3^b from 4 to 4096.
#define FFST_COL_CASES(X) X(4) X(6) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) \
  X(12) X(24) X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)                             \
  X(9) X(18) X(36) X(72) X(144) X(288) X(576) X(1152) X(2304)                               \
  X(27) X(54) X(108) X(216) X(432) X(864) X(1728) X(3456) X(81) X(162) X(324) X(648) X(1296) X(2592)  \
  X(243) X(486) X(972) X(1944) X(3888) X(729) X(1458) X(2916) X(2187)

}  // namespace

bool supported_length(int L) {
  switch (L) {
#define CASE(n) case n: return true;
    FFST_COL_CASES(CASE)
#undef CASE
    default: return false;
  }
}

hipError_t launch_line_fft(int M, float2* F, int nlines, int pitch, bool inverse, const float2* parts, int nparts,
                           long long part_stride, const float2* twM, hipStream_t s) {
  if (nlines == 0) return hipSuccess;
  switch (M) {
#define CASE(n)                                                                                        \
  case n:                                                                                              \
    if constexpr (alt_col_values(n) != 0)                                                             \
      if (alt_cols_requested(n))                                                                       \
        return line_fft_with<n, alt_col_values(n)>(F, nlines, pitch, inverse, parts, nparts, part_stride, twM, s); \
    return line_fft_with<n, 0>(F, nlines, pitch, inverse, parts, nparts, part_stride, twM, s);
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd_cols(const FwdColArgs& a, hipStream_t s) {
  FwdColJob job{a.F, a.psic, a.col_ptr, a.col_planes, a.col_hull, a.N / 2 + 1, a.nimg, std::max(a.nparts, 1),
                a.pitch, a.win, a.y_img_stride, a.y_off_base, a.Y, a.scale, a.twM};
  if (job.nimg == 0) return hipSuccess;
  const long long total = (long long)job.H * job.nimg * job.nparts;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n:                                                                                         \
    if constexpr (alt_col_values(n) != 0)                                                        \
      if (alt_cols_requested(n)) return fwd_cols_with<n, alt_col_values(n)>(job, total, s);      \
    return fwd_cols_with<n, 0>(job, total, s);
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_lines(const AdjLineArgs& a, hipStream_t s) {
  AdjLineJob job{a.Z, a.z_img_stride, a.z_off_base, a.win, a.psic, a.col_ptr, a.col_planes, a.col_hull,
                 a.N / 2 + 1, a.nimg, a.nparts, a.pitch, a.accumulate, a.out, a.scale, a.twM};
  if (job.nimg == 0) return hipSuccess;
  const long long total = (long long)job.H * job.nimg * job.nparts;
  switch (a.M) {
#define CASE(n)                                                                                   \
  case n:                                                                                         \
    if constexpr (alt_col_values(n) != 0)                                                        \
      if (alt_cols_requested(n)) return adj_lines_with<n, alt_col_values(n)>(job, total, a.fused, s); \
    return adj_lines_with<n, 0>(job, total, a.fused, s);
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffst
