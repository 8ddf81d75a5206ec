// launch_cfg.hpp -- lane/row/line shapes of the FFT kernels and the
// persistent-grid sizing shared by the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_core.hpp"

namespace ffst {

// Values per lane for lengths with a factor 3. 3 * 2^k use 12 (radices 12,
// 4, ..., 2; 6 and 3 one stage). 9 * 2^k below 576 use 18 (radices 18, 2,
// ..., 2; 9 itself one radix-9 stage); from 576 on the radix-2 stages of that
// plan need more twiddle registers than a lane has, and 12 values (radices
// 12, 12, 4 ...) take over. Lengths with 27 or a higher power of 3 use 12
// when 4 divides them (radices 12, ..., then 6 or 3 for the remaining
// threes), else 18 or 9 (then 9 and 3). With 12 values a group of 9 * 2^k or
// 27 * 2^k lanes is not a power of two wide.
__host__ __device__ constexpr int values_with_three(int L) {
  return (L % 9 == 0 && L % 4 == 0 && (L % 27 == 0 || L >= 576)) ? 12
         : L % 9 == 0 ? (L % 2 == 0 ? 18 : 9)
                      : (L >= 12 ? 12 : L);
}

// Values per lane along rows: 16 for powers of two from 16 on.
__host__ __device__ constexpr int line_values(int L) {
  return L % 3 == 0 ? values_with_three(L) : (L >= 16 ? 16 : L);
}
// Column lines: 8 values per lane below length 1024 (8*8*8 needs the same
// two exchanges as 16*16*2 for 512, with far fewer registers), 16 from 1024
// on (one wave per line at 1024, measured faster than 8 values on two waves);
// lengths with a factor 3 as along rows.
__host__ __device__ constexpr int col_values(int L) {
  return L % 3 == 0 ? values_with_three(L) : (L >= 1024 ? 16 : (L >= 8 ? 8 : L));
}

// Rows per block that divide the image height: all M rows when M < rb_max,
// else the largest divisor of M that divides rb_max (rb_max is a power of two).
inline int rows_per_block(int M, int rb_max) {
  if (M < rb_max) return M;
  int rb = rb_max;
  while (M % rb) rb /= 2;
  return rb;
}

// Index helpers for lengths that need not be powers of two.
__device__ __forceinline__ int wrap_once(int x, int L) { return x >= L ? x - L : x; }   // x in [0, 2L)
__device__ __forceinline__ int mirror_index(int r, int L) { return r == 0 ? 0 : L - r; }  // -r mod L, r in [0, L)

// LDS stride per line/row: congruent to 17 mod 32, so that 16 lanes reading
// the same column of 16 rows, and 16 lanes reading 16 consecutive values of
// one row, both touch distinct banks.
__host__ __device__ constexpr int lds_stride(int L, int V) { return stride_mod32(lds_group_len(L, V), 17); }

__host__ __device__ constexpr int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
__host__ __device__ constexpr int pow2_floor(int x) {
  int p = 1;
  while (2 * p <= x) p *= 2;
  return p;
}

// Lane slots of a group of G lanes. Groups of up to 64 lanes take the next
// power of two of slots, so that groups tile wavefronts and exchange through
// LDS with wave-level ordering only; wider groups (block barriers) take
// exactly G. In a padded group the spare lanes act as copies of lane G - 1
// (group_lane): the same loads, the same arithmetic, and the same values
// stored to the same addresses in the same instructions.
__host__ __device__ constexpr int group_slots(int G) { return G <= 64 ? pow2_ceil(G) : G; }

template <class C>
__device__ __forceinline__ int group_index() {
  return threadIdx.x / C::GS;
}
template <class C>
__device__ __forceinline__ int group_lane() {
  const int j = threadIdx.x % C::GS;
  return C::GS == C::G ? j : min(j, C::G - 1);
}

// Rows per block of the row kernels: 16 (128-byte column segments in the
// transposed phase) while that keeps a block at <= 512 threads, whose 256
// registers per lane hold a pipelined row FFT without spilling; longer rows
// take fewer rows per block (512 / GS, rounded down to a power of two).
__host__ __device__ constexpr int row_block_rows(int GS) {
  return GS <= 16 ? 256 / GS : (GS <= 32 ? 16 : pow2_floor(512 / GS));
}

// Tunable launch shapes (set per call from the plan, read by the launchers):
// the values per lane of the column-line FFTs (0: col_values(M); otherwise
// alt_col_values(M), where compiled) and the height of the row blocks (1:
// row_block_rows; 2: alt_block_rows, where compiled).
inline thread_local int t_col_values = 0;
inline thread_local int t_row_block = 1;

// The second lane width compiled for column lines of length L: 16 for the
// powers of two that use 8 (and 8 where 16 is the default), 6 for 3 * 2^k
// from 96 on (radix 6 then 2s, against 12 then 4s); 0 where none is.
__host__ __device__ constexpr int alt_col_values(int L) {
  return (L & (L - 1)) == 0 ? (L >= 64 ? (L >= 1024 ? 8 : 16) : 0)
                            : ((L % 3 == 0 && L % 9 != 0 && L >= 96 && ((L / 3) & (L / 3 - 1)) == 0) ? 6 : 0);
}

// Row lengths L (complex length N/2) whose kernels are also compiled with
// the alternative row-block height: powers of two and 3 * 2^k from 32 on.
__host__ __device__ constexpr bool row_block_tunable(int L) {
  return L >= 32 && (((L & (L - 1)) == 0) || (L % 3 == 0 && ((L / 3) & (L / 3 - 1)) == 0));
}

// The alternative row-block height: twice the default for rows of up to 16
// lane slots (a 512-thread block), half of it for wider rows, whose default
// block has 512 threads already (doubling would cap the registers at 128 and
// spill).
__host__ __device__ constexpr int alt_block_rows(int GS) {
  return GS <= 16 ? 2 * row_block_rows(GS) : (row_block_rows(GS) >= 2 ? row_block_rows(GS) / 2 : 1);
}

// Real rows of length N = 2L (complex FFT of length L), RB rows per block
// (RBM = 2: the alternative height). Rows of 1024 and 2048 points take 32
// values per lane. 2048 (radix 32 x 32): 32 lanes per row, so a 512-thread
// block holds 16 rows and writes 128-byte column segments (with 16 values:
// 8 rows, 64 bytes; measured 0.73 -> 0.65 ms for the inverse row pass of a
// 2048 x 2048 image). 1024 (radix 32 x 16): one LDS exchange instead of two
// (16 x 16 x 2) and 256-thread blocks of 16 rows (the 64-image uneven batch:
// 6.15 -> 5.94 ms). Longer rows would spill with 32 values.
template <int L, int RBM = 1>
struct RowCfg {
  static constexpr int V = (L == 512 || L == 1024) ? 32 : line_values(L);
  static constexpr int G = L / V;                      // lanes per row
  static constexpr int GS = group_slots(G);            // lane slots per row
  static constexpr int SYNC = GS <= 64 ? kWave : kBlock;
  static constexpr int RB = RBM == 2 ? alt_block_rows(GS) : row_block_rows(GS);
  static constexpr int THREADS = RB * GS;
  static constexpr int STRIDE = lds_stride(L, V);
  // wave-level sync needs groups that tile wavefronts exactly
  static_assert(SYNC == kBlock || (GS & (GS - 1)) == 0, "row slots must be a power of two");
  static_assert(THREADS <= 1024, "row block too large");
};

// Complex rows of length L (complex FFT of length L), RB rows per block.
template <int L>
struct CRowCfg {
  static constexpr int V = line_values(L);
  static constexpr int G = L / V;
  static constexpr int GS = group_slots(G);
  static constexpr int SYNC = GS <= 64 ? kWave : kBlock;
  static constexpr int RB = row_block_rows(GS);
  static constexpr int THREADS = RB * GS;
  static constexpr int STRIDE = lds_stride(L, V);
  static_assert(SYNC == kBlock || (GS & (GS - 1)) == 0, "row slots must be a power of two");
  static_assert(THREADS <= 1024, "row block too large");
};

// Contiguous lines of length L (the column direction, L = M); VV != 0
// replaces the default values per lane.
template <int L, int VV = 0>
struct LineCfg {
  static constexpr int V = VV ? VV : col_values(L);
  static constexpr int G = L / V;
  static constexpr int GS = group_slots(G);
  static constexpr int SYNC = GS <= 64 ? kWave : kBlock;
  static constexpr int THREADS = GS <= 64 ? 256 : GS;  // kBlock: one line per block
  static constexpr int LPB = THREADS / GS;             // lines per block
  static constexpr int STRIDE = lds_stride(L, V);
  // groups must tile wavefronts and the block exactly
  static_assert((SYNC == kBlock || (GS & (GS - 1)) == 0) && LPB * GS == THREADS, "line slots must tile the block");
  static_assert(THREADS <= 1024, "line block too large");
};

// Compute units of the current device (read once per process; the static's
// initialisation is thread-safe).
inline int num_cus() {
  static const int n = [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        prop.multiProcessorCount > 0)
      return prop.multiProcessorCount;
    return 256;
  }();
  return n;
}

// Persistent blocks per CU for the launches of the current call on this
// thread (0: the per-kernel default below); set from a plan's tuning.
inline thread_local int t_blocks_per_cu = 0;

// Persistent grids: enough blocks for the work, at most `per_cu` per CU.
inline int grid_for(long long units, int threads) {
  const int per_cu = t_blocks_per_cu > 0 ? t_blocks_per_cu : (threads >= 1024 ? 2 : (threads >= 512 ? 4 : 8));
  const long long cap = (long long)num_cus() * per_cu;
  return (int)(units < cap ? (units > 0 ? units : 1) : cap);
}

// Loads of data that is read once and not soon again (the coefficients of a
// large batch): non-temporal, so they stream past the caches instead of
// evicting the intermediates the next kernel reads back.
__device__ __forceinline__ float2 load_stream(const float2* p) {
  const unsigned long long b = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
  float2 v;
  __builtin_memcpy(&v, &b, sizeof v);
  return v;
}

__device__ __forceinline__ float load_stream(const float* p) { return __builtin_nontemporal_load(p); }

// Reads above this size (about half the 256 MB Infinity Cache) use load_stream.
constexpr long long kStreamBytes = 128LL << 20;

// Rows per block for a launch over `units_of_planes` planes of M rows: the
// fixed block height, halved (down to 4 rows, and only while the half still
// divides M) while the launch would have fewer blocks than CUs.
inline int rows_per_launch(int M, int rb_max, long long units_of_planes) {
  int rb = rows_per_block(M, rb_max);
  while (rb > 4 && rb % 2 == 0 && M % (rb / 2) == 0 && units_of_planes * (M / rb) < num_cus()) rb /= 2;
  return rb;
}

// A unit of the row kernels: rows r0 .. r0 + rb - 1 of plane `plane` of
// image `img`; units run image-major, then plane, then row block.
struct RowUnit {
  int img, plane, r0;
};

__device__ __forceinline__ RowUnit row_unit(int u, int blocks_per_plane, int nplanes, float inv_nplanes, int rb,
                                            int plane0) {
  RowUnit ru;
  const int pq = u / blocks_per_plane;
  ru.r0 = (u - pq * blocks_per_plane) * rb;
  ru.img = (int)(((float)pq + 0.5f) * inv_nplanes);  // exact for pq < 2^20
  ru.plane = plane0 + pq - ru.img * nplanes;
  return ru;
}

}  // namespace ffst
