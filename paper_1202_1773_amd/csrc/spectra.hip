// spectra.hip -- shearlet spectra on the frequency grid, evaluated in float64
// on the device and stored in float32 (run once per plan).
//
// Grid (Sec. 3.5.1): omega_1 = Delta * q_N(c) along columns, omega_2 =
// Delta * q_M(r) along rows, q_D(p) = p for p <= ceil(D/2) - 1 and p - D
// otherwise (natural DFT order). Only the half plane c = 0 .. N/2 is stored,
// column-contiguous: psi[i][c][r] (the layout the column passes stream).
//
// Windows (Sec. 2.1, 2.4, 3.4):
//   v(x)      = x^4 (35 - 84 x + 70 x^2 - 20 x^3) on [0, 1], clamped outside
//               (or one of the other choices of the Remark on the construction
//               of v: C^k polynomials, C-infinity)
//   psi1(w)   = 0 | sin(pi/2 v(2|w|-1)) | 1 | cos(pi/2 v(|w|/2-1)) | 0 on the
//               breakpoints 1/2, 1, 2, 4 (the closed form of Sec. 3.4)
//   psi2(w)   = sqrt(v(1 - |w|))
//   varphi(w) = 1 | cos(pi/2 v(2|w|-1)) | 0 on the breakpoints 1/2, 1
// Spectra (Sec. 3.1, eq. shearletTransform):
//   low-pass  varphi(max(|w1|, |w2|))                           (eq. phi)
//   (h, j, k) psi1(4^-j w1) psi2(2^j w2/w1 + k)  where |w2| < |w1|
//   (v, j, k) psi1(4^-j w2) psi2(2^j w1/w2 + k)  where |w1| < |w2|
//   seam      h formula where |w2| <= |w1| (w1 != 0), v formula elsewhere
// Smooth variant (Sec. 3.4, eq. newPsi1, eq. smoothPsi): psi1(4^-j w_a) is
// replaced by sqrt(Phi^2(w/4^(j+1)) - Phi^2(w/4^j)) with the tensor low-pass
// Phi(w) = varphi(w1) varphi(w2) (eq. Phi), which is also the low-pass.
// Real coefficients (Sec. 3.8.1): on the Nyquist column (N even) the value at
// row r and the value at row -r mod M are both replaced by their root mean
// square; on the Nyquist row (M even) likewise for columns c and -c mod N.
#include "internal.hpp"

#include <math.h>

namespace ffst {
namespace {

// Auxiliary function v on [0, 1], clamped outside. aux = 3: eq. (v) by
// Horner; aux = k >= 1: the C^k choice v'(x) = c x^k (x-1)^k, v(1) = 1, i.e.
// the binomial tail sum_{m=k+1}^{2k+1} C(2k+1, m) x^m (1-x)^(2k+1-m) (every
// term nonnegative), summed upward with the ratio of consecutive terms;
// aux < 0: the C-infinity choice s(x-1) / (s(x-1) + s(x)) of the Remark on
// the construction of v, written as 1 / (1 + s(x) / s(x-1)) so that neither
// exponential underflows into 0/0.
__device__ double v_aux(double x, int aux) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  if (aux == 3) {
    const double x2 = x * x;
    return x2 * x2 * (35.0 + x * (-84.0 + x * (70.0 - 20.0 * x)));
  }
  if (aux < 0) {
    const double e_lo = 1.0 / (x * x) + 1.0 / ((2.0 - x) * (2.0 - x));          // -log s(x - 1)
    const double e_hi = 1.0 / ((1.0 + x) * (1.0 + x)) + 1.0 / ((1.0 - x) * (1.0 - x));  // -log s(x)
    return 1.0 / (1.0 + exp(e_lo - e_hi));
  }
  const int n = 2 * aux + 1;
  const double y = 1.0 - x;
  double binom = 1.0;                      // C(n, k + 1)
  for (int m = 1; m <= aux + 1; ++m) binom = binom * (double)(n - m + 1) / (double)m;
  double term = binom * pow(x, (double)(aux + 1)) * pow(y, (double)aux);
  double sum = 0.0;
  for (int m = aux + 1; m <= n; ++m) {
    sum += term;
    term *= (double)(n - m) / (double)(m + 1) * (x / y);
  }
  return sum;
}

__device__ double psi1_hat(double w, int aux) {
  const double a = fabs(w);
  if (a <= 0.5) return 0.0;
  if (a < 1.0) return sin(M_PI_2 * v_aux(2.0 * a - 1.0, aux));
  if (a <= 2.0) return 1.0;
  if (a < 4.0) return cos(M_PI_2 * v_aux(0.5 * a - 1.0, aux));
  return 0.0;
}

__device__ double psi2_hat(double w, int aux) { return sqrt(v_aux(1.0 - fabs(w), aux)); }

__device__ double varphi(double w, int aux) {
  const double a = fabs(w);
  if (a <= 0.5) return 1.0;
  if (a < 1.0) return cos(M_PI_2 * v_aux(2.0 * a - 1.0, aux));
  return 0.0;
}

// Smooth corona function of Sec. 3.4 at the dilated point 4^-j w.
__device__ double corona(double w1, double w2, double dil, int aux) {
  const double a1 = w1 * dil, a2 = w2 * dil;
  const double outer = varphi(0.25 * a1, aux) * varphi(0.25 * a2, aux);
  const double inner = varphi(a1, aux) * varphi(a2, aux);
  const double d = outer * outer - inner * inner;
  return d > 0.0 ? sqrt(d) : 0.0;
}

__device__ double spectrum_value(int kind, int j, int k, int smooth, int aux, double w1, double w2) {
  const double a1 = fabs(w1), a2 = fabs(w2);
  if (kind == KIND_LOWPASS) {
    if (smooth) return varphi(w1, aux) * varphi(w2, aux);
    return a2 <= a1 ? varphi(w1, aux) : varphi(w2, aux);
  }
  const double dil = ldexp(1.0, -2 * j);   // 4^-j
  const double shr = ldexp(1.0, j);        // 2^j
  const bool use_v = (kind == KIND_V) ? (a1 < a2) : (kind == KIND_SEAM && a1 < a2);
  const bool use_h = (kind == KIND_H) ? (a2 < a1) : (kind == KIND_SEAM && !(a1 < a2) && a1 > 0.0);
  if (use_h) {
    const double radial = smooth ? corona(w1, w2, dil, aux) : psi1_hat(w1 * dil, aux);
    return radial == 0.0 ? 0.0 : radial * psi2_hat(shr * (w2 / w1) + k, aux);
  }
  if (use_v) {
    const double radial = smooth ? corona(w1, w2, dil, aux) : psi1_hat(w2 * dil, aux);
    return radial == 0.0 ? 0.0 : radial * psi2_hat(shr * (w1 / w2) + k, aux);
  }
  return 0.0;
}

__device__ __forceinline__ int signed_freq(int p, int D) { return p <= (D + 1) / 2 - 1 ? p : p - D; }

__device__ double grid_value(const GenParams& g, int kind, int j, int k, int r, int c) {
  const double w1 = g.delta * signed_freq(c, g.N);
  const double w2 = g.delta * signed_freq(r, g.M);
  return spectrum_value(kind, j, k, g.smooth, g.aux, w1, w2);
}

// Grid value with the real-coefficient fix of Sec. 3.8.1, at any point
// (r, c) of the full plane.
__device__ double fixed_value(const GenParams& g, int kd, int j, int k, int r, int c) {
  double val = grid_value(g, kd, j, k, r, c);
  if (g.N % 2 == 0 && c == g.N / 2) {
    const double b = grid_value(g, kd, j, k, (g.M - r) % g.M, c);
    val = sqrt(0.5 * (val * val + b * b));
  } else if (g.M % 2 == 0 && r == g.M / 2) {
    const double b = grid_value(g, kd, j, k, r, (g.N - c) % g.N);
    val = sqrt(0.5 * (val * val + b * b));
  }
  return val;
}

__global__ void __launch_bounds__(256) k_spectra(GenParams g, const int* __restrict__ kind,
                                                 const int* __restrict__ jj, const int* __restrict__ kk,
                                                 float* __restrict__ psi) {
  const int H = g.N / 2 + 1;
  const long long n = (long long)g.M * H;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (idx >= n) return;
  const int c = (int)(idx / g.M), r = (int)(idx % g.M);
  psi[(long long)i * n + idx] = (float)fixed_value(g, kind[i], jj[i], kk[i], r, c);
}

// First and last half-plane column holding a nonzero value, per plane:
// one block per (column, plane) line.
__global__ void __launch_bounds__(256) k_windows(const float* __restrict__ psi, int M, int H,
                                                 int* __restrict__ lo, int* __restrict__ hi) {
  const int c = blockIdx.x;
  const int i = blockIdx.y;
  const float* p = psi + ((long long)i * H + c) * M;
  int any = 0;
  for (int r = threadIdx.x; r < M; r += blockDim.x) any |= (p[r] != 0.0f);
  if (__syncthreads_or(any) && threadIdx.x == 0) {
    atomicMin(lo + i, c);
    atomicMax(hi + i, c);
  }
}

// Row-major copy of the spectra: out[i][r][c] for c < cols (cols = N/2 + 1,
// or N with the missing columns filled by evenness on the grid).
__global__ void __launch_bounds__(256) k_expand(const float* __restrict__ psi, int M, int N, int cols,
                                                float* __restrict__ out) {
  const int H = N / 2 + 1;
  const long long n = (long long)M * cols;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (idx >= n) return;
  const int r = (int)(idx / cols), c = (int)(idx % cols);
  const int rr = c < H ? r : (M - r) % M;
  const int cc = c < H ? c : N - c;
  out[(long long)i * n + idx] = psi[((long long)i * H + cc) * M + rr];
}

// ---- one-sided spectra (Sec. 3.8.2) ----
//
// Spectrum i >= 1 is centred on the ray of direction d = (1, -k / 2^j) in
// (omega_1, omega_2) (h cone and seam elements) or d = (-k / 2^j, 1) (v cone).
// Its one-sided version keeps the lobe on the side <omega, d> > 0, scaled by
// sqrt(2), and drops the other; where a grid point and its DFT mirror are not
// on opposite sides (the line <omega, d> = 0, and pairs on a Nyquist line)
// the value is kept as is. The sign of <omega, d> is taken on the integer
// frequencies: with one spacing Delta for both axes it is the sign of
// 2^j q_N(c) - k q_M(r) (h, seam) or 2^j q_M(r) - k q_N(c) (v).
__device__ int side_sign(int kd, int j, int k, int r, int c, int M, int N) {
  const long long n1 = signed_freq(c, N), n2 = signed_freq(r, M);
  const long long s = kd == KIND_V ? (-(long long)k * n1 + ((long long)1 << j) * n2)
                                   : (((long long)1 << j) * n1 - (long long)k * n2);
  return (s > 0) - (s < 0);
}

__device__ double one_sided_factor(int kd, int j, int k, int r, int c, int M, int N) {
  if (kd == KIND_LOWPASS) return 1.0;
  const int sd = side_sign(kd, j, k, r, c, M, N);
  if (sd == 0 || side_sign(kd, j, k, (M - r) % M, (N - c) % N, M, N) != -sd) return 1.0;
  return sd > 0 ? M_SQRT2 : 0.0;
}

// flags[i][c] = 1 if column c (full plane, c < N) of the one-sided spectrum i
// holds a nonzero value; one block per (column, spectrum). Reads the
// half-plane spectra (even on the grid: Psi(r, c) = Psi(-r, -c)).
__global__ void __launch_bounds__(256) k_one_sided_flags(const float* __restrict__ psi, int M, int N,
                                                         const int* __restrict__ kind, const int* __restrict__ jj,
                                                         const int* __restrict__ kk, unsigned char* __restrict__ flags) {
  const int c = blockIdx.x;
  const int i = blockIdx.y;
  const int H = N / 2 + 1;
  const int kd = kind[i], j = jj[i], k = kk[i];
  const bool upper = c >= H;
  const float* p = psi + ((long long)i * H + (upper ? N - c : c)) * M;
  int any = 0;
  for (int r = threadIdx.x; r < M; r += blockDim.x) {
    const float v = p[upper ? (M - r) % M : r];
    any |= (v != 0.0f && one_sided_factor(kd, j, k, r, c, M, N) != 0.0);
  }
  const int all = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[(long long)i * N + c] = all ? 1 : 0;
}

// Compact one-sided spectra: plane i holds w[i] columns of M values starting
// at psip + poff[i]; column m is the full-plane column (lo[i] + m) mod N.
__global__ void __launch_bounds__(256) k_one_sided_pack(GenParams g, const int* __restrict__ kind,
                                                        const int* __restrict__ jj, const int* __restrict__ kk,
                                                        const int* __restrict__ lo, const int* __restrict__ w,
                                                        const long long* __restrict__ poff, float* __restrict__ psip) {
  const int i = blockIdx.y;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)w[i] * g.M) return;
  const int m = (int)(idx / g.M), r = (int)(idx % g.M);
  const int c = (lo[i] + m) % g.N;
  const int kd = kind[i], j = jj[i], k = kk[i];
  const double val = one_sided_factor(kd, j, k, r, c, g.M, g.N) * fixed_value(g, kd, j, k, r, c);
  psip[poff[i] + idx] = (float)val;
}

// Row-major full-plane copy of the compact one-sided spectra.
__global__ void __launch_bounds__(256) k_one_sided_expand(const float* __restrict__ psip, int M, int N,
                                                          const int* __restrict__ lo, const int* __restrict__ w,
                                                          const long long* __restrict__ poff, float* __restrict__ out) {
  const long long n = (long long)M * N;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (idx >= n) return;
  const int r = (int)(idx / N), c = (int)(idx % N);
  const int m = ((c - lo[i]) % N + N) % N;
  out[(long long)i * n + idx] = m < w[i] ? psip[poff[i] + (long long)m * M + r] : 0.0f;
}

}  // namespace

hipError_t launch_one_sided_flags(const float* psi, int M, int N, int eta, const int* kind, const int* jj,
                                  const int* kk, unsigned char* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_one_sided_flags, dim3((unsigned)N, (unsigned)eta), dim3(256), 0, s, psi, M, N, kind, jj, kk,
                     flags);
  return hipGetLastError();
}

hipError_t launch_one_sided_pack(const GenParams& g, int eta, int max_w, const int* kind, const int* jj,
                                 const int* kk, const int* lo, const int* w, const long long* poff, float* psip,
                                 hipStream_t s) {
  const long long n = (long long)max_w * g.M;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_one_sided_pack, dim3((unsigned)((n + 255) / 256), (unsigned)eta), dim3(256), 0, s, g, kind,
                     jj, kk, lo, w, poff, psip);
  return hipGetLastError();
}

hipError_t launch_one_sided_expand(const float* psip, int M, int N, int eta, const int* lo, const int* w,
                                   const long long* poff, float* out, hipStream_t s) {
  const long long n = (long long)M * N;
  hipLaunchKernelGGL(k_one_sided_expand, dim3((unsigned)((n + 255) / 256), (unsigned)eta), dim3(256), 0, s, psip, M,
                     N, lo, w, poff, out);
  return hipGetLastError();
}

hipError_t launch_spectra(const GenParams& g, int eta, const int* kind, const int* jj, const int* kk,
                          float* psi, hipStream_t s) {
  const long long n = (long long)g.M * (g.N / 2 + 1);
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)eta);
  hipLaunchKernelGGL(k_spectra, grid, dim3(256), 0, s, g, kind, jj, kk, psi);
  return hipGetLastError();
}

hipError_t launch_windows(const float* psi, int M, int N, int eta, int* lo, int* hi, hipStream_t s) {
  const int H = N / 2 + 1;
  dim3 grid((unsigned)H, (unsigned)eta);
  hipLaunchKernelGGL(k_windows, grid, dim3(256), 0, s, psi, M, H, lo, hi);
  return hipGetLastError();
}

hipError_t launch_expand(const float* psi, int M, int N, int eta, int cols, float* out, hipStream_t s) {
  const long long n = (long long)M * cols;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)eta);
  hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, s, psi, M, N, cols, out);
  return hipGetLastError();
}

}  // namespace ffst
