// Device-side FFT building blocks for gfx950: self-sorting (Stockham) radix
// 2/3/4/8 passes over transforms held in LDS, complex helpers, and the
// compile-time radix plan.  A transform of length L is processed by T = L/P
// threads, each owning P points per pass (P divisible by every radix used).
//
// Stockham pass with radix R and span p (product of the radices already
// applied), for butterfly i in [0, L/R), k = i mod p:
//     u_r = a[i + r L/R] * w^(r k / (p R)),  r = 0..R-1,  w = exp(-+2 pi i)
//     U   = DFT_R(u)
//     b[(i - k) R + k + r p] = U_r
// After the last pass the data are in natural order.
#pragma once
#include <hip/hip_runtime.h>

namespace rihvr {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Small DFTs, X_q = sum_m x_m exp(-+2 pi i m q / R)  (sign + for INV)
// ---------------------------------------------------------------------------
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV> struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float c = -0.5f, s = 0.86602540378443864676f;  // cos, sin of 2 pi / 3
    float2 s12 = cadd(v[1], v[2]);
    float2 d12 = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x + c * s12.x, v[0].y + c * s12.y);
    // forward: X1 = m - i s d, X2 = m + i s d
    float2 isd = INV ? make_float2(-s * d12.y, s * d12.x) : make_float2(s * d12.y, -s * d12.x);
    v[0] = cadd(v[0], s12);
    v[1] = cadd(m, isd);
    v[2] = csub(m, isd);
  }
};

template <bool INV> struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV> struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // twiddles exp(-+ i pi q / 4), q = 1..3
    float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                    : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    float2 o2 = mul_mi<INV>(o[2]);
    float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                    : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// ---------------------------------------------------------------------------
// Compile-time radix plan.  L = 2^a or 3 * 2^a.  A radix-3 pass comes first,
// then radix 8 while it divides both the remaining length and P, then 4 / 2.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int next_radix(int rem, int P) {
  return (rem % 3 == 0) ? 3
       : (rem % 8 == 0 && P % 8 == 0) ? 8
       : (rem % 4 == 0 && P % 4 == 0) ? 4
       : 2;
}

__host__ __device__ constexpr bool valid_len(int L) {
  int n = L;
  if (n % 3 == 0) n /= 3;
  while (n % 2 == 0) n /= 2;
  return n == 1;
}

// Points per thread for a transform of length L.
__host__ __device__ constexpr int points_per_thread(int L) {
  return (L % 3 == 0) ? (L >= 12 ? 12 : L) : (L >= 8 ? 8 : L);
}

// Ordering point between the LDS writes and reads of a transform: a block
// barrier, or, when each transform lies inside one wavefront (WAVE), only an
// ordering of that wave's LDS accesses (the LDS executes one wave's operations
// in issue order), so that waves holding different transforms never wait for
// each other.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham pass.  `buf` holds the transform with element e at buf[e*S].
// `tw` is a table exp(-2 pi i m / (L*TWS)), m in [0, L*TWS), read with stride TWS.
template <int R, int L, int P, int S, int TWS, int p, bool INV, bool WAVE>
__device__ __forceinline__ void stockham_pass(float2* buf, int t, const float2* __restrict__ tw) {
  constexpr int T = L / P;
  constexpr int NB = P / R;
  static_assert(P % R == 0, "radix must divide the points per thread");
  float2 v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + b * T;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = buf[(i + r * (L / R)) * S];
  }
  lds_sync<WAVE>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + b * T;
    const int k = i % p;
    if (p > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[(r * k * (L / (p * R))) * TWS];
        v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
      }
    }
    Dft<R, INV>::run(v[b]);
    const int j = (i - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(j + r * p) * S] = v[b][r];
  }
  lds_sync<WAVE>();
}

template <int L, int P, int S, int TWS, int p, int rem, bool INV, bool WAVE>
__device__ __forceinline__ void stockham_rest(float2* buf, int t, const float2* __restrict__ tw) {
  if constexpr (rem > 1) {
    constexpr int R = next_radix(rem, P);
    stockham_pass<R, L, P, S, TWS, p, INV, WAVE>(buf, t, tw);
    stockham_rest<L, P, S, TWS, p * R, rem / R, INV, WAVE>(buf, t, tw);
  }
}

// Full in-LDS transform of length L (unscaled).  Every thread of the block (of
// the wave, with WAVE) must call it; thread t in [0, L/P) of each transform
// owns P points per pass.
template <int L, int P, int S, int TWS, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_lds(float2* buf, int t, const float2* __restrict__ tw) {
  static_assert(valid_len(L), "length must be 2^a or 3*2^a");
  stockham_rest<L, P, S, TWS, 1, L, INV, WAVE>(buf, t, tw);
}

}  // namespace rihvr
