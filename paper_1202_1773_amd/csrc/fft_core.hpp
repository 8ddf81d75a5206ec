// fft_core.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A length-L transform is carried by a "group" of G = L / V lanes; every lane
// holds V complex values in registers, lane j holding element j + G*s in slot
// s (s = 0 .. V-1). That layout is the same before and after the transform,
// so a group loads and stores with unit stride across lanes (coalesced for
// rows, tile-interleaved for columns).
//
// Each stage is a radix-R Stockham autosort step (R = V, and one final
// smaller radix when L is not a power of V). A lane runs V/R butterflies per
// stage; butterfly b reads elements b + t*L/R, twiddles them by
// W_{pR}^{t (b mod p)} (p = product of the earlier radices), applies the
// R-point DFT in registers and writes element (b/p)*p*R + (b mod p) + t*p.
// Between stages the values travel through LDS; after the last stage they
// are back in the lane layout above, in natural order. Twiddles come from a
// table tw[m] = exp(-2 pi i m / (L*ts)) (float32, rounded from float64 on the
// host), read with stride ts.
//
// Every thread of the block must call these functions the same number of
// times (they contain block barriers).
#pragma once

#include <hip/hip_runtime.h>

namespace ffst {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// a * (-i) for the forward direction, a * (+i) for the inverse.
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// a * exp(-+ i pi / 4)
template <bool INV>
__device__ __forceinline__ float2 rot45(float2 a) {
  constexpr float c = 0.70710678118654752440f;
  return INV ? make_float2((a.x - a.y) * c, (a.x + a.y) * c)
             : make_float2((a.x + a.y) * c, (a.y - a.x) * c);
}

// a * exp(-+ 3 i pi / 4)
template <bool INV>
__device__ __forceinline__ float2 rot135(float2 a) {
  constexpr float c = 0.70710678118654752440f;
  return INV ? make_float2(-(a.x + a.y) * c, (a.x - a.y) * c)
             : make_float2((a.y - a.x) * c, -(a.x + a.y) * c);
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  static __device__ __forceinline__ void run(float2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
  }
};

template <bool INV>
struct Dft<4, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    float2 t2 = cadd(a[1], a[3]), t3 = rot90<INV>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[4] = {a[0], a[2], a[4], a[6]};
    float2 o[4] = {a[1], a[3], a[5], a[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    o[1] = rot45<INV>(o[1]);
    o[2] = rot90<INV>(o[2]);
    o[3] = rot135<INV>(o[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 4] = csub(e[k], o[k]);
    }
  }
};

template <bool INV>
struct Dft<16, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = a[2 * k];
      o[k] = a[2 * k + 1];
    }
    Dft<8, INV>::run(e);
    Dft<8, INV>::run(o);
    // o[k] *= exp(-+ 2 pi i k / 16)
    constexpr float c1 = 0.92387953251128675613f;  // cos(pi/8)
    constexpr float s1 = 0.38268343236508977173f;  // sin(pi/8)
    const float sg = INV ? 1.0f : -1.0f;
    o[1] = cmul(o[1], make_float2(c1, sg * s1));
    o[2] = rot45<INV>(o[2]);
    o[3] = cmul(o[3], make_float2(s1, sg * c1));
    o[4] = rot90<INV>(o[4]);
    o[5] = cmul(o[5], make_float2(-s1, sg * c1));
    o[6] = rot135<INV>(o[6]);
    o[7] = cmul(o[7], make_float2(-c1, sg * s1));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 8] = csub(e[k], o[k]);
    }
  }
};

// LDS index with one padding slot per 8 complex values (spreads the
// power-of-two strides of the Stockham writes over the banks).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_len(int L) { return L + (L >> 3) + 1; }

template <int L, int V, int R, int P, bool LAST, bool INV>
__device__ __forceinline__ void stockham_stage(float2 (&u)[V], int j, float2* lds,
                                               const float2* __restrict__ tw, int ts) {
  constexpr int G = L / V;
  constexpr int NB = V / R;
  constexpr int TSTEP = L / (P * R);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    const int b = j + m * G;
    const int k = b % P;
    float2 a[R];
#pragma unroll
    for (int t = 0; t < R; ++t) a[t] = u[m + t * NB];
    if constexpr (P > 1) {
#pragma unroll
      for (int t = 1; t < R; ++t) {
        float2 w = tw[(t * k * TSTEP) * ts];
        if constexpr (INV) w.y = -w.y;
        a[t] = cmul(a[t], w);
      }
    }
    Dft<R, INV>::run(a);
    if constexpr (LAST) {
#pragma unroll
      for (int t = 0; t < R; ++t) u[m + t * NB] = a[t];
    } else {
      const int base = (b / P) * P * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) lds[lpad(base + t * P)] = a[t];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < V; ++s) u[s] = lds[lpad(j + G * s)];
    __syncthreads();
  }
}

template <int L, int V, int P, bool INV>
struct Stages {
  static __device__ __forceinline__ void run(float2 (&u)[V], int j, float2* lds,
                                             const float2* __restrict__ tw, int ts) {
    constexpr int REM = L / P;
    constexpr int R = (REM % V == 0) ? V : REM;
    static_assert(V % R == 0, "final radix must divide the values per lane");
    constexpr bool LAST = (P * R == L);
    stockham_stage<L, V, R, P, LAST, INV>(u, j, lds, tw, ts);
    if constexpr (!LAST) Stages<L, V, P * R, INV>::run(u, j, lds, tw, ts);
  }
};

// In-place length-L FFT of the group's values (forward: kernel exp(-2 pi i nk/L),
// inverse: exp(+2 pi i nk/L), both unnormalised).
template <int L, int V, bool INV>
__device__ __forceinline__ void fft_group(float2 (&u)[V], int j, float2* lds,
                                          const float2* __restrict__ tw, int ts) {
  Stages<L, V, 1, INV>::run(u, j, lds, tw, ts);
}

// Values per lane used for a transform of length L.
__host__ __device__ constexpr int values_per_lane(int L) { return L >= 2048 ? 16 : (L >= 8 ? 8 : L); }

}  // namespace ffst
