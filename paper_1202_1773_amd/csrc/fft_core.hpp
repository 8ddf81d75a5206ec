// fft_core.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A length-L transform is carried by a "group" of G = L / V lanes; every lane
// holds V complex values in registers, lane j holding element j + G*s in slot
// s (s = 0 .. V-1). That layout is the same before and after the transform,
// so a group loads and stores with unit stride across lanes.
//
// Each stage is a radix-R Stockham autosort step, R being the largest
// divisor of V that divides what is left of L (V, V, ..., then a smaller
// power of two; with V = 12 for lengths 3 * 2^k: 12, 4, ..., 4, 2; with
// V = 18 for lengths 9 * 2^k: 18, 2, ..., 2). A lane
// runs V/R butterflies per
// stage; butterfly b reads elements b + t*L/R, multiplies them by the twiddles
// W_{pR}^{t (b mod p)} (p = product of the earlier radices), applies the
// R-point DFT in registers and writes element (b/p)*p*R + (b mod p) + t*p.
// Between stages the values travel through LDS; after the last stage they
// are back in the lane layout above, in natural order.
//
// The twiddles a lane needs depend only on its lane index j, so they are read
// once from a float32 table (rounded from float64 on the host) into
// registers (TwiddleRegs) and reused for every transform the lane runs.
//
// Exchange synchronisation: when the whole group sits inside one wavefront
// (Sync = kWave) the exchange only needs the LDS accesses of the wave to stay
// in program order, which the hardware guarantees; a compiler barrier keeps
// the compiler from reordering them. Otherwise (Sync = kBlock) block barriers
// are used and every thread of the block must call the transform the same
// number of times.
#pragma once

#include <hip/hip_runtime.h>

namespace ffst {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
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

// sin(pi/3), cos(pi/6)
constexpr float kSin60 = 0.86602540378443864676f;

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
struct Dft<3, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    // y1,2 = a0 - (a1 + a2)/2 -+ i sin(2 pi/3) (a1 - a2) (forward sign)
    const float2 t = cadd(a[1], a[2]);
    const float2 m = make_float2(a[0].x - 0.5f * t.x, a[0].y - 0.5f * t.y);
    const float2 d = csub(a[1], a[2]);
    const float2 s = rot90<INV>(make_float2(kSin60 * d.x, kSin60 * d.y));
    a[0] = cadd(a[0], t);
    a[1] = cadd(m, s);
    a[2] = csub(m, s);
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
    constexpr float sg = INV ? 1.0f : -1.0f;
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

// 32 = 2 x 16: DFT16 of the even and the odd elements, twiddles
// exp(-+ 2 pi i k / 32), k < 16.
template <bool INV>
struct Dft<32, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[16], o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      e[k] = a[2 * k];
      o[k] = a[2 * k + 1];
    }
    Dft<16, INV>::run(e);
    Dft<16, INV>::run(o);
    // cos(k pi / 16), k = 0 .. 8
    constexpr float c[9] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f, 0.83146961230254523708f,
                            0.70710678118654752440f, 0.55557023301960222474f, 0.38268343236508977173f,
                            0.19509032201612826785f, 0.0f};
    constexpr float sg = INV ? 1.0f : -1.0f;
#pragma unroll
    for (int k = 1; k < 16; ++k) {
      // exp(-+ i k pi / 16) = (cos, -+ sin), sin(k pi/16) = cos((8 - k) pi/16)
      const float ck = k <= 8 ? c[k] : -c[16 - k];
      const float sk = k <= 8 ? c[8 - k] : c[k - 8];
      o[k] = cmul(o[k], make_float2(ck, sg * sk));
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 16] = csub(e[k], o[k]);
    }
  }
};

// 6 = 2 x 3: DFT3 of the even and the odd elements, twiddles exp(-+ 2 pi i k / 6).
template <bool INV>
struct Dft<6, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[3] = {a[0], a[2], a[4]};
    float2 o[3] = {a[1], a[3], a[5]};
    Dft<3, INV>::run(e);
    Dft<3, INV>::run(o);
    constexpr float sg = INV ? 1.0f : -1.0f;
    o[1] = cmul(o[1], make_float2(0.5f, sg * kSin60));
    o[2] = cmul(o[2], make_float2(-0.5f, sg * kSin60));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 3] = csub(e[k], o[k]);
    }
  }
};

// 12 = 2 x 6, twiddles exp(-+ 2 pi i k / 12).
template <bool INV>
struct Dft<12, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[6], o[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      e[k] = a[2 * k];
      o[k] = a[2 * k + 1];
    }
    Dft<6, INV>::run(e);
    Dft<6, INV>::run(o);
    constexpr float sg = INV ? 1.0f : -1.0f;
    o[1] = cmul(o[1], make_float2(kSin60, sg * 0.5f));
    o[2] = cmul(o[2], make_float2(0.5f, sg * kSin60));
    o[3] = rot90<INV>(o[3]);
    o[4] = cmul(o[4], make_float2(-0.5f, sg * kSin60));
    o[5] = cmul(o[5], make_float2(-kSin60, sg * 0.5f));
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 6] = csub(e[k], o[k]);
    }
  }
};

// cos and sin of 20, 40 and 80 degrees (the ninth and eighteenth roots of unity)
constexpr float kCos20 = 0.93969262078590838405f, kSin20 = 0.34202014332566873304f;
constexpr float kCos40 = 0.76604444311897803520f, kSin40 = 0.64278760968653932632f;
constexpr float kCos80 = 0.17364817766693034885f, kSin80 = 0.98480775301220805936f;

// 9 = 3 x 3: DFT3 over a[n2], a[n2+3], a[n2+6] for each n2, twiddles
// exp(-+ 2 pi i n2 k1 / 9), then DFT3 over n2 giving outputs k1, k1+3, k1+6.
template <bool INV>
struct Dft<9, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    constexpr float sg = INV ? 1.0f : -1.0f;
    float2 t[3][3];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
      t[n2][0] = a[n2];
      t[n2][1] = a[n2 + 3];
      t[n2][2] = a[n2 + 6];
      Dft<3, INV>::run(t[n2]);
    }
    t[1][1] = cmul(t[1][1], make_float2(kCos40, sg * kSin40));   // w^1
    t[1][2] = cmul(t[1][2], make_float2(kCos80, sg * kSin80));   // w^2
    t[2][1] = cmul(t[2][1], make_float2(kCos80, sg * kSin80));   // w^2
    t[2][2] = cmul(t[2][2], make_float2(-kCos20, sg * kSin20));  // w^4 (160 degrees)
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      float2 u[3] = {t[0][k1], t[1][k1], t[2][k1]};
      Dft<3, INV>::run(u);
      a[k1] = u[0];
      a[k1 + 3] = u[1];
      a[k1 + 6] = u[2];
    }
  }
};

// 18 = 2 x 9, twiddles exp(-+ 2 pi i k / 18) = exp(-+ i k 20 degrees).
template <bool INV>
struct Dft<18, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 e[9], o[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      e[k] = a[2 * k];
      o[k] = a[2 * k + 1];
    }
    Dft<9, INV>::run(e);
    Dft<9, INV>::run(o);
    constexpr float sg = INV ? 1.0f : -1.0f;
    o[1] = cmul(o[1], make_float2(kCos20, sg * kSin20));
    o[2] = cmul(o[2], make_float2(kCos40, sg * kSin40));
    o[3] = cmul(o[3], make_float2(0.5f, sg * kSin60));
    o[4] = cmul(o[4], make_float2(kCos80, sg * kSin80));
    o[5] = cmul(o[5], make_float2(-kCos80, sg * kSin80));
    o[6] = cmul(o[6], make_float2(-0.5f, sg * kSin60));
    o[7] = cmul(o[7], make_float2(-kCos40, sg * kSin40));
    o[8] = cmul(o[8], make_float2(-kCos20, sg * kSin20));
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      a[k] = cadd(e[k], o[k]);
      a[k + 9] = csub(e[k], o[k]);
    }
  }
};

// ----------------------------------------------------------- radix plan

// Largest divisor of V that divides n.
__host__ __device__ constexpr int largest_common_radix(int V, int n) {
  int r = 1;
  for (int d = 1; d <= V; ++d)
    if (V % d == 0 && n % d == 0) r = d;
  return r;
}

// Radices for length L with V values per lane: at each stage the largest
// divisor of V that divides the remaining length (V, V, ..., then a smaller
// one; every radix divides V).
template <int L, int V>
struct RadixPlan {
  static_assert(L % V == 0, "V must divide L");
  static constexpr int G = L / V;
  static constexpr int radix(int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= largest_common_radix(V, L / p);
    return largest_common_radix(V, L / p);
  }
  static constexpr int span(int s) {  // product of the radices before stage s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= radix(i);
    return p;
  }
  static constexpr int stages() {
    int n = 0;
    for (int p = 1; p < L; p *= radix(n), ++n) {
    }
    return n;
  }
  // offset of stage s's twiddles inside the per-lane register table
  static constexpr int tw_offset(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += (V / radix(i)) * (radix(i) - 1);
    return o;
  }
  static constexpr int NTW = tw_offset(stages());
};

// Per-lane twiddles of all stages after the first (forward sign; the inverse
// uses the conjugates). table[m] = exp(-2 pi i m / (L * ts)).
template <int L, int V>
struct TwiddleRegs {
  using P = RadixPlan<L, V>;
  float2 w[P::NTW > 0 ? P::NTW : 1];

  template <int S>
  __device__ __forceinline__ void load_stage(int j, const float2* __restrict__ table, int ts) {
    if constexpr (S < P::stages()) {
      constexpr int R = P::radix(S), SP = P::span(S), NB = V / R, TSTEP = L / (SP * R);
      constexpr int OFF = P::tw_offset(S);
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const int k = (j + m * P::G) % SP;
#pragma unroll
        for (int t = 1; t < R; ++t) w[OFF + m * (R - 1) + t - 1] = table[(t * k * TSTEP) * ts];
      }
      load_stage<S + 1>(j, table, ts);
    }
  }
  // The lane index passes through an empty asm first, so the optimizer does
  // not use its known range here: with that range (lane = threadIdx % G) the
  // compiler of this toolchain produced wrong twiddles for length 144 with 18
  // values per lane (measured on gfx950; the same code with threadIdx was
  // correct). The load runs once per kernel.
  __device__ __forceinline__ void load(int j, const float2* __restrict__ table, int ts) {
    __asm__ __volatile__("" : "+v"(j));
    load_stage<1>(j, table, ts);
  }
  // Multiplies a[1 .. R-1] of butterfly m of stage S by their twiddles.
  template <int S, int R, bool INV>
  __device__ __forceinline__ void apply(float2 (&a)[R], int m) const {
    constexpr int OFF = P::tw_offset(S);
#pragma unroll
    for (int t = 1; t < R; ++t) {
      const float2 x = w[OFF + m * (R - 1) + t - 1];
      a[t] = INV ? cmulc(a[t], x) : cmul(a[t], x);
    }
  }
};

// The same twiddles with one register pair per butterfly instead of R - 1:
// only w = table[k * TSTEP] is kept, and w^t (t = 2 .. R-1) is rebuilt at
// every use by squaring and one more product (w^2t = (w^t)^2,
// w^(2t+1) = w^2t * w), at most 2 log2(R) roundings away from the table
// value. The seed passes through an empty asm at each use, so the compiler
// cannot hoist the powers out of the caller's loops back into registers.
// For kernels whose occupancy is set by their registers and whose vector ALU
// has time to spare.
template <int L, int V>
struct TwiddleSeeds {
  using P = RadixPlan<L, V>;
  static constexpr int seed_offset(int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += V / P::radix(i);
    return o;
  }
  static constexpr int NSEED = seed_offset(P::stages());
  float2 w[NSEED > 0 ? NSEED : 1];

  template <int S>
  __device__ __forceinline__ void load_stage(int j, const float2* __restrict__ table, int ts) {
    if constexpr (S < P::stages()) {
      constexpr int R = P::radix(S), SP = P::span(S), NB = V / R, TSTEP = L / (SP * R);
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const int k = (j + m * P::G) % SP;
        w[seed_offset(S) + m] = table[(k * TSTEP) * ts];
      }
      load_stage<S + 1>(j, table, ts);
    }
  }
  // The lane index passes through an empty asm, as in TwiddleRegs::load
  // (without it the length-144 kernels compute wrong twiddles).
  __device__ __forceinline__ void load(int j, const float2* __restrict__ table, int ts) {
    __asm__ __volatile__("" : "+v"(j));
    load_stage<1>(j, table, ts);
  }
  template <int S, int R, bool INV>
  __device__ __forceinline__ void apply(float2 (&a)[R], int m) const {
    float2 p[R];
    p[1] = w[seed_offset(S) + m];
    __asm__ __volatile__("" : "+v"(p[1].x), "+v"(p[1].y));
#pragma unroll
    for (int t = 2; t < R; ++t) p[t] = (t % 2 == 0) ? cmul(p[t / 2], p[t / 2]) : cmul(p[t - 1], p[1]);
#pragma unroll
    for (int t = 1; t < R; ++t) a[t] = INV ? cmulc(a[t], p[t]) : cmul(a[t], p[t]);
  }
};

enum SyncKind { kWave = 0, kBlock = 1 };

template <int SYNC>
__device__ __forceinline__ void lds_sync() {
  if constexpr (SYNC == kBlock) {
    __syncthreads();
  } else {
    // LDS accesses of one wavefront complete in program order; only the
    // compiler has to be kept from moving them across this point.
    __builtin_amdgcn_wave_barrier();
    __asm__ __volatile__("" ::: "memory");
  }
}

// LDS index with one padding slot per V complex values.
template <int V>
__device__ __forceinline__ int lpad(int i) {
  return i + i / V;
}

template <int L, int V, int S, bool INV, int SYNC, class TW>
__device__ __forceinline__ void stockham_stage(float2 (&u)[V], int j, float2* lds, const TW& tw) {
  using P = RadixPlan<L, V>;
  constexpr int G = P::G, R = P::radix(S), SP = P::span(S), NB = V / R;
  constexpr bool LAST = (S + 1 == P::stages());
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    float2 a[R];
#pragma unroll
    for (int t = 0; t < R; ++t) a[t] = u[m + t * NB];
    if constexpr (S > 0) tw.template apply<S, R, INV>(a, m);
    Dft<R, INV>::run(a);
    if constexpr (LAST) {
#pragma unroll
      for (int t = 0; t < R; ++t) u[m + t * NB] = a[t];
    } else {
      const int b = j + m * G;
      const int base = (b / SP) * SP * R + (b % SP);
#pragma unroll
      for (int t = 0; t < R; ++t) lds[lpad<V>(base + t * SP)] = a[t];
    }
  }
  if constexpr (!LAST) {
    lds_sync<SYNC>();
#pragma unroll
    for (int s = 0; s < V; ++s) u[s] = lds[lpad<V>(j + G * s)];
    lds_sync<SYNC>();
    stockham_stage<L, V, S + 1, INV, SYNC>(u, j, lds, tw);
  }
}

// In-place length-L FFT of the group's values (forward: kernel exp(-2 pi i nk/L),
// inverse: exp(+2 pi i nk/L), both unnormalised). TW is TwiddleRegs<L, V> or
// TwiddleSeeds<L, V>.
template <int L, int V, bool INV, int SYNC, class TW>
__device__ __forceinline__ void fft_group(float2 (&u)[V], int j, float2* lds, const TW& tw) {
  stockham_stage<L, V, 0, INV, SYNC>(u, j, lds, tw);
}

// Complex elements of LDS a group needs (padded indices stay below this).
__host__ __device__ constexpr int lds_group_len(int L, int V) { return L + L / V + 1; }

// Smallest stride >= n that is congruent to r modulo 32 (in complex elements);
// used to spread the groups of one half-wavefront over all LDS banks.
__host__ __device__ constexpr int stride_mod32(int n, int r) { return n + ((r - n % 32) % 32 + 32) % 32; }

}  // namespace ffst
