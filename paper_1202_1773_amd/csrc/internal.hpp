// internal.hpp -- declarations shared by the host code and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ffst {

// Spectrum kinds, one per index i (Sec. 3.5.2 order is built on the host).
enum SpecKind : int { KIND_LOWPASS = 0, KIND_H = 1, KIND_V = 2, KIND_SEAM = 3 };

struct GenParams {
  int M, N;
  double delta;       // grid spacing (Sec. 3.5.1)
  int smooth;         // 0: Meyer shearlets, 1: smooth shearlets of Sec. 3.4
};

// Per-plane nonzero column window [lo, lo + w) of the half plane and the
// plane's offset (in complex elements) inside one image's compact buffer.
struct Windows {
  const int* lo;
  const int* w;
  const long long* off;
};

// Kernel ids for timing (must match kKernelNames in api.hip).
enum KernelId : int {
  KID_SPECTRA = 0,
  KID_WINDOWS,
  KID_R2C_IMAGE,
  KID_FFT_COLS_IMAGE,
  KID_FWD_COLS,
  KID_C2R_PLANES,
  KID_R2C_PLANES,
  KID_ADJ_COLS,
  KID_IFFT_COLS_IMAGE,
  KID_C2R_IMAGE,
  KID_EXPAND,
  KID_COUNT
};

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_spectra(const GenParams& g, int eta, const int* kind, const int* jj, const int* kk,
                          float* psi, hipStream_t s);
hipError_t launch_windows(const float* psi, int M, int N, int eta, int* lo, int* hi, hipStream_t s);
hipError_t launch_expand(const float* psi, int M, int N, int eta, int cols, float* out, hipStream_t s);

// Row transforms of length N = 2L. The rows of a unit are (img, plane, r) for
// img < nimg, plane0 <= plane < plane0 + nplanes, r < M; real row
// (img, plane, r) starts at x + img*x_img_stride + (plane*M + r)*N. The
// complex side is column-contiguous: column c of (img, plane) holds M values
// at z + img*z_img_stride + (win.off[plane] - z_off_base) + (c - lo)*zp, for
// the half-plane columns c in [lo, lo + w) of the plane's window.
struct RowArgs {
  float* x;
  float2* z;
  long long x_img_stride, z_img_stride, z_off_base;
  int nimg, nplanes, plane0, M, N;
  int zp;                   // complex elements between consecutive columns of z
  Windows win;
  const float2* twN;
};
hipError_t launch_r2c_rows(const RowArgs& a, hipStream_t s);
hipError_t launch_c2r_rows(const RowArgs& a, hipStream_t s);

// In-place FFT of nlines contiguous lines of length M; the inverse may first
// replace each line by the sum of the same line in `nparts` partial arrays.
hipError_t launch_line_fft(int M, float2* F, int nlines, int pitch, bool inverse, const float2* parts, int nparts,
                           long long part_stride, const float2* twM, hipStream_t s);

struct FwdLineArgs {
  int M, N;
  const float2* F;          // [nimg][N/2+1][M]
  const float* psi;         // [eta][N/2+1][M]
  const int2* lines;        // (spectrum, column)
  int nlines, nimg;
  int pitch;                // complex elements between column lines of F and Y
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};
hipError_t launch_fwd_lines(const FwdLineArgs& a, hipStream_t s);

struct AdjLineArgs {
  int M, N;
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psi;
  const int* col_ptr;
  const int* col_planes;
  int nimg, nparts, accumulate, fused;
  int pitch;                // complex elements between column lines of Z, A and partial sums
  float2* out;
  float scale;
  const float2* twM;
};
hipError_t launch_adj_lines(const AdjLineArgs& a, hipStream_t s);

bool supported_length(int L);

}  // namespace ffst
