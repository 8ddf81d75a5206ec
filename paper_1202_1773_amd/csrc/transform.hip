// transform.hip -- the FFST hot path on gfx950.
//
// Forward (eq. shearletTransform): F = fft2(f) as a real-to-complex row pass
// (k_r2c_rows) and an in-place column pass (k_fft_cols_image); then, per
// spectrum i and tile of half-plane columns, k_fwd_cols loads the tile of F,
// multiplies by Psi_i / (M N), runs the inverse column FFT and stores the
// tile into a compact per-plane intermediate Y_i that only spans the
// columns where Psi_i is nonzero; k_c2r_rows finishes each row with a
// complex-to-real inverse FFT and writes the coefficients. Psi_i * F is never
// stored.
//
// Adjoint / inverse (eq. inverseShearletTransform): k_r2c_rows on every
// coefficient row, keeping only the columns inside Psi_i's window (Z_i);
// k_adj_cols loads, per tile of columns, the Z_i of every spectrum touching
// the tile, runs the forward column FFT, multiplies by Psi_i and accumulates
// in registers (the sum over (j, k)), then applies the inverse column FFT to
// the sum; k_c2r_rows turns the result into the image.
//
// Real FFT of length N = 2L along a row: z[n] = x[2n] + i x[2n+1],
// Z = FFT_L(z), X[k] = ((Z[k] + conj Z[L-k]) - i W_N^k (Z[k] - conj Z[L-k])) / 2
// for k = 0 .. L. Its inverse forms Z'[k] = (X[k] + conj X[L-k]) +
// i W_N^-k (X[k] - conj X[L-k]), applies the unnormalised inverse FFT_L and
// reads x[2n] = Re, x[2n+1] = Im; that is the unnormalised length-N inverse
// DFT of the Hermitian row.
#include "fft_core.hpp"
#include "internal.hpp"

namespace ffst {
namespace {

constexpr int kRowBlock = 256;

template <int L>
struct RowCfg {
  static constexpr int V = values_per_lane(L);
  static constexpr int G = L / V;
  static constexpr int RB = kRowBlock / G;  // rows per block
  static_assert(G <= kRowBlock, "row too long");
};

template <int M>
struct ColCfg {
  static constexpr int V = values_per_lane(M);
  static constexpr int G = M / V;
  static constexpr int TW = (8 * G <= 1024) ? 8 : 1024 / G;  // columns per tile
  static constexpr int THREADS = TW * G;
};

// ---------------------------------------------------------------- rows

template <int L>
__global__ void __launch_bounds__(kRowBlock) k_r2c_rows(const float* __restrict__ x, long long nrows, int M,
                                                        int planes, float2* __restrict__ out,
                                                        long long img_stride, Windows win,
                                                        const float2* __restrict__ twN) {
  using C = RowCfg<L>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::RB * lds_len(L)];
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  const long long row = (long long)blockIdx.x * C::RB + g;
  const bool valid = row < nrows;
  float2* my = lds + g * lds_len(L);

  float2 u[V];
  const float2* xr = reinterpret_cast<const float2*>(x) + (valid ? row : 0) * (long long)L;
#pragma unroll
  for (int s = 0; s < V; ++s) u[s] = valid ? xr[j + G * s] : make_float2(0.f, 0.f);

  fft_group<L, V, false>(u, j, my, twN, 2);

  // Z[L - k] for every k held by this lane.
#pragma unroll
  for (int s = 0; s < V; ++s) my[lpad(j + G * s)] = u[s];
  __syncthreads();
  float2 zm[V];
#pragma unroll
  for (int s = 0; s < V; ++s) zm[s] = my[lpad((L - (j + G * s)) % L)];
  __syncthreads();

  if (!valid) return;
  const int r = (int)(row % M);
  const long long pr = row / M;
  const int p = (int)(pr % planes);
  const long long img = pr / planes;
  const int lo = win.lo[p], w = win.w[p];
  float2* o = out + img * img_stride + win.off[p] + (long long)r * w;
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = j + G * s;
    if (k >= lo && k < lo + w) {
      const float2 zc = conjf2(zm[s]);
      const float2 a = cadd(u[s], zc);
      const float2 b = cmul(twN[k], csub(u[s], zc));
      o[k - lo] = cscale(csub(a, make_float2(-b.y, b.x)), 0.5f);
    }
  }
  if (j == 0 && L >= lo && L < lo + w) o[L - lo] = make_float2(u[0].x - u[0].y, 0.f);
}

template <int L>
__global__ void __launch_bounds__(kRowBlock) k_c2r_rows(const float2* __restrict__ in, long long img_stride,
                                                        Windows win, long long nrows, int M, int planes,
                                                        float* __restrict__ y, float scale,
                                                        const float2* __restrict__ twN) {
  using C = RowCfg<L>;
  constexpr int V = C::V, G = C::G;
  __shared__ float2 lds[C::RB * lds_len(L)];
  const int g = threadIdx.x / G;
  const int j = threadIdx.x % G;
  const long long row = (long long)blockIdx.x * C::RB + g;
  const bool valid = row < nrows;
  float2* my = lds + g * lds_len(L);

  int lo = 0, w = 0;
  const float2* ir = in;
  if (valid) {
    const int r = (int)(row % M);
    const long long pr = row / M;
    const int p = (int)(pr % planes);
    const long long img = pr / planes;
    lo = win.lo[p];
    w = win.w[p];
    ir = in + img * img_stride + win.off[p] + (long long)r * w;
  }
  float2 u[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const int k = j + G * s;
    const int km = L - k;
    const float2 xk = (k >= lo && k < lo + w) ? ir[k - lo] : make_float2(0.f, 0.f);
    const float2 xm = (km >= lo && km < lo + w) ? ir[km - lo] : make_float2(0.f, 0.f);
    const float2 xc = conjf2(xm);
    const float2 a = cadd(xk, xc);
    const float2 b = cmul(conjf2(twN[k]), csub(xk, xc));
    u[s] = cadd(a, make_float2(-b.y, b.x));
  }

  fft_group<L, V, true>(u, j, my, twN, 2);

  if (!valid) return;
  float2* yr = reinterpret_cast<float2*>(y) + row * (long long)L;
#pragma unroll
  for (int s = 0; s < V; ++s) yr[j + G * s] = cscale(u[s], scale);
}

// ------------------------------------------------------------- columns

// F[b] (M x H, H = N/2 + 1) in place: forward FFT along each column.
template <int M>
__global__ void __launch_bounds__(ColCfg<M>::THREADS) k_fft_cols_image(float2* __restrict__ F, int H,
                                                                       const float2* __restrict__ twM) {
  using C = ColCfg<M>;
  constexpr int V = C::V, G = C::G, TW = C::TW;
  __shared__ float2 lds[TW * lds_len(M)];
  const int col = threadIdx.x % TW;
  const int j = threadIdx.x / TW;
  const int c = blockIdx.x * TW + col;
  const bool valid = c < H;
  float2* base = F + (long long)blockIdx.y * M * H + c;
  float2 u[V];
#pragma unroll
  for (int s = 0; s < V; ++s) u[s] = valid ? base[(long long)(j + G * s) * H] : make_float2(0.f, 0.f);
  fft_group<M, V, false>(u, j, lds + col * lds_len(M), twM, 1);
  if (!valid) return;
#pragma unroll
  for (int s = 0; s < V; ++s) base[(long long)(j + G * s) * H] = u[s];
}

// One (image, spectrum, column tile) per block: Y_i = ifft_col(Psi_i * scale * F).
template <int M>
__global__ void __launch_bounds__(ColCfg<M>::THREADS) k_fwd_cols(const float2* __restrict__ F,
                                                                 const float* __restrict__ psi, int H,
                                                                 int batch, const int2* __restrict__ items,
                                                                 Windows win, long long img_stride,
                                                                 float2* __restrict__ Y, float scale,
                                                                 const float2* __restrict__ twM) {
  using C = ColCfg<M>;
  constexpr int V = C::V, G = C::G, TW = C::TW;
  __shared__ float2 lds[TW * lds_len(M)];
  const int col = threadIdx.x % TW;
  const int j = threadIdx.x / TW;
  const int item = blockIdx.x / batch;
  const int b = blockIdx.x % batch;
  const int2 it = items[item];  // (spectrum, first column of the tile)
  const int i = it.x;
  const int c = it.y + col;
  const int lo = win.lo[i], w = win.w[i];
  const bool valid = c < lo + w;
  const float2* fb = F + (long long)b * M * H + c;
  const float* pb = psi + (long long)i * M * H + c;
  float2 u[V];
#pragma unroll
  for (int s = 0; s < V; ++s) {
    const long long off = (long long)(j + G * s) * H;
    u[s] = valid ? cscale(fb[off], pb[off] * scale) : make_float2(0.f, 0.f);
  }
  fft_group<M, V, true>(u, j, lds + col * lds_len(M), twM, 1);
  if (!valid) return;
  float2* yb = Y + (long long)b * img_stride + win.off[i] + (c - lo);
#pragma unroll
  for (int s = 0; s < V; ++s) yb[(long long)(j + G * s) * w] = u[s];
}

// One (image, column tile) per block: A = scale * ifft_col( sum_i Psi_i * fft_col(Z_i) ).
template <int M>
__global__ void __launch_bounds__(ColCfg<M>::THREADS) k_adj_cols(const float2* __restrict__ Z,
                                                                 long long img_stride, Windows win,
                                                                 const float* __restrict__ psi, int H,
                                                                 int batch, const int* __restrict__ tile_ptr,
                                                                 const int* __restrict__ tile_planes,
                                                                 float2* __restrict__ A, float scale,
                                                                 const float2* __restrict__ twM) {
  using C = ColCfg<M>;
  constexpr int V = C::V, G = C::G, TW = C::TW;
  __shared__ float2 lds[TW * lds_len(M)];
  const int col = threadIdx.x % TW;
  const int j = threadIdx.x / TW;
  const int tile = blockIdx.x / batch;
  const int b = blockIdx.x % batch;
  const int c = tile * TW + col;
  const bool in_plane = c < H;
  float2* my = lds + col * lds_len(M);
  float2 acc[V];
#pragma unroll
  for (int s = 0; s < V; ++s) acc[s] = make_float2(0.f, 0.f);

  const int p0 = tile_ptr[tile], p1 = tile_ptr[tile + 1];
  for (int q = p0; q < p1; ++q) {
    const int i = tile_planes[q];
    const int lo = win.lo[i], w = win.w[i];
    const bool valid = in_plane && c >= lo && c < lo + w;
    const float2* zb = Z + (long long)b * img_stride + win.off[i] + (c - lo);
    float2 u[V];
#pragma unroll
    for (int s = 0; s < V; ++s) u[s] = valid ? zb[(long long)(j + G * s) * w] : make_float2(0.f, 0.f);
    fft_group<M, V, false>(u, j, my, twM, 1);
    const float* pb = psi + (long long)i * M * H + c;
#pragma unroll
    for (int s = 0; s < V; ++s) {
      const float ps = valid ? pb[(long long)(j + G * s) * H] : 0.f;
      acc[s].x += ps * u[s].x;
      acc[s].y += ps * u[s].y;
    }
  }
#pragma unroll
  for (int s = 0; s < V; ++s) acc[s] = cscale(acc[s], scale);
  fft_group<M, V, true>(acc, j, my, twM, 1);
  if (!in_plane) return;
  float2* ab = A + (long long)b * M * H + c;
#pragma unroll
  for (int s = 0; s < V; ++s) ab[(long long)(j + G * s) * H] = acc[s];
}

// ------------------------------------------------------------ dispatch

// Row kernels take the complex length L = N/2, column kernels the length M.
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

int col_tile_width(int M) {
  switch (M) {
#define CASE(n) case n: return ColCfg<n>::TW;
    FFST_COL_CASES(CASE)
#undef CASE
    default: return 0;
  }
}

hipError_t launch_r2c_rows(int N, const float* x, long long nrows, int M, int planes, float2* out,
                           long long img_stride, Windows win, const float2* twN, hipStream_t s) {
  const int L = N / 2;
  switch (L) {
#define CASE(n)                                                                                      \
  case n: {                                                                                          \
    const long long blocks = (nrows + RowCfg<n>::RB - 1) / RowCfg<n>::RB;                            \
    hipLaunchKernelGGL(k_r2c_rows<n>, dim3((unsigned)blocks), dim3(kRowBlock), 0, s, x, nrows, M,   \
                       planes, out, img_stride, win, twN);                                          \
    return hipGetLastError();                                                                        \
  }
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_c2r_rows(int N, const float2* in, long long img_stride, Windows win, long long nrows,
                           int M, int planes, float* y, float scale, const float2* twN, hipStream_t s) {
  const int L = N / 2;
  switch (L) {
#define CASE(n)                                                                                      \
  case n: {                                                                                          \
    const long long blocks = (nrows + RowCfg<n>::RB - 1) / RowCfg<n>::RB;                            \
    hipLaunchKernelGGL(k_c2r_rows<n>, dim3((unsigned)blocks), dim3(kRowBlock), 0, s, in, img_stride,\
                       win, nrows, M, planes, y, scale, twN);                                       \
    return hipGetLastError();                                                                        \
  }
    FFST_ROW_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fft_cols_image(int M, int N, float2* F, int batch, const float2* twM, hipStream_t s) {
  const int H = N / 2 + 1;
  switch (M) {
#define CASE(n)                                                                                      \
  case n: {                                                                                          \
    dim3 grid((unsigned)((H + ColCfg<n>::TW - 1) / ColCfg<n>::TW), (unsigned)batch);                \
    hipLaunchKernelGGL(k_fft_cols_image<n>, grid, dim3(ColCfg<n>::THREADS), 0, s, F, H, twM);        \
    return hipGetLastError();                                                                        \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fwd_cols(int M, int N, const float2* F, const float* psi, int batch, const int2* items,
                           int nitems, Windows win, long long img_stride, float2* Y, float scale,
                           const float2* twM, hipStream_t s) {
  const int H = N / 2 + 1;
  switch (M) {
#define CASE(n)                                                                                      \
  case n: {                                                                                          \
    dim3 grid((unsigned)((long long)nitems * batch));                                                \
    hipLaunchKernelGGL(k_fwd_cols<n>, grid, dim3(ColCfg<n>::THREADS), 0, s, F, psi, H, batch, items, \
                       win, img_stride, Y, scale, twM);                                              \
    return hipGetLastError();                                                                        \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adj_cols(int M, int N, const float2* Z, long long img_stride, Windows win,
                           const float* psi, int batch, const int* tile_ptr, const int* tile_planes,
                           int ntiles, float2* A, float scale, const float2* twM, hipStream_t s) {
  const int H = N / 2 + 1;
  switch (M) {
#define CASE(n)                                                                                      \
  case n: {                                                                                          \
    dim3 grid((unsigned)((long long)ntiles * batch));                                                \
    hipLaunchKernelGGL(k_adj_cols<n>, grid, dim3(ColCfg<n>::THREADS), 0, s, Z, img_stride, win, psi, \
                       H, batch, tile_ptr, tile_planes, A, scale, twM);                              \
    return hipGetLastError();                                                                        \
  }
    FFST_COL_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ffst
