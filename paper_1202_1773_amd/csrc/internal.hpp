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
  KID_C2R_IMAGE,
  KID_EXPAND,
  KID_COUNT
};

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_spectra(const GenParams& g, int eta, const int* kind, const int* jj, const int* kk,
                          float* psi, hipStream_t s);
hipError_t launch_windows(const float* psi, int M, int N, int eta, int* lo, int* hi, hipStream_t s);
hipError_t launch_expand(const float* psi, int M, int N, int eta, float* out, hipStream_t s);

// Row transforms of length N = 2L along contiguous rows.
// rows are enumerated as ((img * planes) + p) * M + r.
hipError_t launch_r2c_rows(int N, const float* x, long long nrows, int M, int planes, float2* out,
                           long long img_stride, Windows win, const float2* twN, hipStream_t s);
hipError_t launch_c2r_rows(int N, const float2* in, long long img_stride, Windows win, long long nrows,
                           int M, int planes, float* y, float scale, const float2* twN, hipStream_t s);

// Column transforms of length M over the half plane (N/2 + 1 columns).
hipError_t launch_fft_cols_image(int M, int N, float2* F, int batch, const float2* twM, hipStream_t s);
hipError_t launch_fwd_cols(int M, int N, const float2* F, const float* psi, int batch, const int2* items,
                           int nitems, Windows win, long long img_stride, float2* Y, float scale,
                           const float2* twM, hipStream_t s);
hipError_t launch_adj_cols(int M, int N, const float2* Z, long long img_stride, Windows win,
                           const float* psi, int batch, const int* tile_ptr, const int* tile_planes,
                           int ntiles, float2* A, float scale, const float2* twM, hipStream_t s);

// Columns per column-kernel tile for a transform length M.
int col_tile_width(int M);
bool supported_length(int L);

}  // namespace ffst
