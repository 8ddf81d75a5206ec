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
  int aux;            // auxiliary function v: 3 = eq. (v), k >= 1 = C^k, -1 = C-infinity
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
  KID_FWD_COLS,
  KID_C2R_PLANES,
  KID_R2C_PLANES,
  KID_ADJ_COLS,
  KID_IFFT_COLS_IMAGE,
  KID_C2R_IMAGE,
  KID_EXPAND,
  KID_ONE_SIDED,            // one-sided spectra: column flags and packing
  KID_FWD_COLS_C,           // complex path: column lines of the forward
  KID_C2C_PLANES_INV,       //   inverse complex row FFTs writing the coefficients
  KID_C2C_PLANES_FWD,       //   forward complex row FFTs of the coefficients
  KID_ADJ_COLS_C,           //   column lines of the adjoint
  KID_COUNT
};

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_spectra(const GenParams& g, int eta, const int* kind, const int* jj, const int* kk,
                          float* psi, hipStream_t s);
hipError_t launch_windows(const float* psi, int M, int N, int eta, int* lo, int* hi, hipStream_t s);
hipError_t launch_expand(const float* psi, int M, int N, int eta, int cols, float* out, hipStream_t s);
hipError_t launch_one_sided_flags(const float* psi, int M, int N, int eta, const int* kind, const int* jj,
                                  const int* kk, unsigned char* flags, hipStream_t s);
hipError_t launch_one_sided_pack(const GenParams& g, int eta, int max_w, const int* kind, const int* jj,
                                 const int* kk, const int* lo, const int* w, const long long* poff, float* psip,
                                 hipStream_t s);
hipError_t launch_one_sided_expand(const float* psip, int M, int N, int eta, const int* lo, const int* w,
                                   const long long* poff, float* out, hipStream_t s);

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
  const float* sign_scale = nullptr;   // r2c only: read s * sign(x) (device scalar s)
};
hipError_t launch_r2c_rows(const RowArgs& a, hipStream_t s);
hipError_t launch_c2r_rows(const RowArgs& a, hipStream_t s);

// In-place FFT of nlines contiguous lines of length M; the inverse may first
// replace each line by the sum of the same line in `nparts` partial arrays.
hipError_t launch_line_fft(int M, float2* F, int nlines, int pitch, bool inverse, const float2* parts, int nparts,
                           long long part_stride, const float2* twM, hipStream_t s);

// Spectrum column lines over their cyclic nonzero hull: line (i, c) holds
// Psi_i at rows (r_lo + m) mod M, m < K, at psic + off; elsewhere Psi_i is
// zero on that column. A line's hull is the int4 (r_lo, K, off, 0).
//
// Forward column pass: per (column c, image, part), the column FFT of the
// image's row transforms F (not yet transformed along the columns), then for
// every nparts-th spectrum i of the plane group whose window holds c the
// inverse column FFT of Psi_i[c] F[c] / (M N) into Y_i.
struct FwdColArgs {
  int M, N;
  const float2* F;          // row transforms, column-contiguous [nimg][N/2+1][pitch]
  const float* psic;        // compact spectrum lines
  const int* col_ptr;       // CSR of the plane group: column -> spectra
  const int* col_planes;
  const int4* col_hull;     // hull of every CSR entry's line
  int nimg, nparts;         // nparts: lines per column sharing its spectra
  int pitch;                // complex elements between column lines of F and Y
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};
hipError_t launch_fwd_cols(const FwdColArgs& a, hipStream_t s);

struct AdjLineArgs {
  int M, N;
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psic;        // compact spectrum lines (see FwdColArgs)
  const int* col_ptr;
  const int* col_planes;
  const int4* col_hull;     // hull of (col_planes[t], column) for every CSR entry t
  int nimg, nparts, accumulate, fused;
  int pitch;                // complex elements between column lines of Z, A and partial sums
  float2* out;
  float scale;
  const float2* twM;
};
hipError_t launch_adj_lines(const AdjLineArgs& a, hipStream_t s);

// ---- complex (one-sided) shearlets ----
//
// Windows are cyclic ranges of full-plane columns: plane i holds the columns
// (lo[i] + m) mod N for m < w[i]; column m of (img, plane) sits at
// z + img*z_img_stride + (win.off[plane] - z_off_base) + m*zp, and the
// compact one-sided spectrum's column m at psip + poff[plane] + m*M.

// Complex rows of length N; row (img, plane, r) of the coefficients starts
// at x + img*x_img_stride + (plane*M + r)*N (complex elements).
struct CRowArgs {
  float2* x;
  float2* z;
  long long x_img_stride, z_img_stride, z_off_base;
  int nimg, nplanes, plane0, M, N;
  int zp;
  Windows win;
  const float2* twN;
};
// Inverse row FFT of the window columns into full complex rows (unnormalised).
hipError_t launch_c2c_rows_inv(const CRowArgs& a, hipStream_t s);
// Forward row FFT of full complex rows, storing the window columns.
hipError_t launch_c2c_rows_fwd(const CRowArgs& a, hipStream_t s);

struct CFwdColArgs {
  int M, N;
  const float2* F;          // row transforms of the images, half-plane columns [nimg][N/2+1][pitch]
  const float* psic;        // one-sided spectrum lines over their hulls
  const int* col_ptr;       // half-plane column -> entries (CSR of this plane group)
  const int2* col_ent;      // (spectrum, 4 * window column + flags); in each column the
                            // entries with flag 1 or 3 come before those with flag 2
  const int4* col_hull;     // hull (first row, length, offset in psic) of every entry's line
  int nimg, nparts;
  int pitch;
  Windows win;
  long long y_img_stride, y_off_base;
  float2* Y;
  float scale;
  const float2* twM;
};
// Per half-plane column c of every image: column FFT of the row transforms,
// then ifft_col(Psi+_i[m] * scale * X) into Y_i for every entry of the
// column, X being the image spectrum's column c (flags 1, 3) or full-plane
// column N - c (flag 2: conj X(-r) of column c).
hipError_t launch_fwd_cols_c(const CFwdColArgs& a, hipStream_t s);

struct CAdjLineArgs {
  int M, N;
  const float2* Z;
  long long z_img_stride, z_off_base;
  Windows win;
  const float* psic;        // one-sided spectrum lines over their hulls
  const int* col_ptr;       // half-plane column -> entries (CSR of the adjoint)
  const int2* col_ent;      // (spectrum, 4 * window column + flag), flag 1: column c, 2: column N - c
                            // (a column c = N - c appears once with each flag)
  const int4* col_hull;     // hull of every entry's line; for flag 2 that of the reversed line Psi(-r)
  int nimg, nparts, accumulate, fused;
  int pitch;
  float2* out;
  float scale;
  const float2* twM;
};
hipError_t launch_adj_lines_c(const CAdjLineArgs& a, hipStream_t s);

// Device memory of plans and batches (counted for ffst_device_bytes; the
// FFST_FAULT_ALLOC test hook fails the n-th allocation inside one creation
// call, counted from the outermost AllocScope).
hipError_t dev_alloc(void** p, size_t bytes);
void dev_free(void* p);
struct AllocScope {
  AllocScope();
  ~AllocScope();
};

// Error reporting shared by the C ABI files: stores the message returned by
// ffst_last_error on this thread (and writes it to the FFST_LOG log) and
// returns `status`.
int fail(int status, const char* fmt, ...);

// Text log selected by the FFST_LOG environment variable (read once):
// unset, empty or 0 = off; 1 = plans, batches, tuning and errors; 2 = also
// every transform call; "<level>:<path>" or a bare path (level 1) appends to
// that file instead of stderr. Lines are written whole, under a lock.
int log_level();
void log_line(int level, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// roctx range over a scope (shown on rocprofv3 --marker-trace timelines;
// nearly free when no profiler is attached). `name` must outlive the scope.
struct Range {
  explicit Range(const char* name);
  ~Range();
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};
// While set, kernel timing is skipped (launches being captured into a graph).
void profile_suspend(bool on);
}  // namespace ffst

struct ffst_plan;
namespace ffst {
// Workspace bytes a call with `batch` images needs under any tuning setting.
size_t workspace_upper_bound(const ffst_plan* p, int batch);

// Column lengths M and row lengths N the kernels are instantiated for:
// powers of two in [8, 4096] and 3 * 2^k in [12, 3072].
bool supported_length(int M);
bool supported_row_length(int N);

}  // namespace ffst
