// Register-resident line FFTs with compile-time sizes.
//
// A line of N complex points is held by T threads, E = N/T points each.  The
// transform is a Stockham decomposition N = R0 R1 R2 R3 (R = 1 for unused
// stages) in which every radix divides E, so each thread owns whole
// butterflies in every stage: stage s, radix R, span Ns = R0...R_{s-1};
// thread tl owns butterflies j = tl + T c (c < E/R), whose inputs are
// x[j + r N/R] and whose outputs go to y[(j/Ns) Ns R + j%Ns + r Ns] after the
// twiddle W_{Ns R}^{r (j%Ns)}.  Between stages the data crosses LDS once, as
// separate real and imaginary planes of doubles.
//
// Register order: v[c*R + r] is input r of butterfly c of the current stage
// (stage 0: v[r] = x[tl + T r]); after run(), v[c*Rl + r] is output r of
// butterfly c of the last stage, at position tl + T c + r N/Rl (the last
// stage has Ns Rl = N).
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.h"

namespace lmvd {
namespace rf {

// ---- small DFTs in registers -------------------------------------------------

template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(double2*) {}
};
template <int DIR>
struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(double2* v) { small_dft<2, -1>(v); }
};
template <int DIR>
struct Dft<3, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft3<DIR>(v); }
};
template <int DIR>
struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }
};
template <int DIR>
struct Dft<8, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft8<DIR>(v); }
};

constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

// Prime-factor (Good-Thomas) composition for coprime A, B: no inner twiddles.
// x[(n1 B + n2 A) mod AB] -> a[n1][n2]; DFT_B along n2, DFT_A along n1;
// X[(k1 B tB + k2 A tA) mod AB] = a[k1][k2], tB = B^{-1} mod A, tA = A^{-1} mod B.
template <int A, int B, int DIR>
__device__ __forceinline__ void dft_pfa(double2* v) {
  constexpr int N = A * B;
  constexpr int tB = inv_mod(B % A, A), tA = inv_mod(A % B, B);
  double2 a[A][B];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1)
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) a[n1][n2] = v[(n1 * B + n2 * A) % N];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) Dft<B, DIR>::run(a[n1]);
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    double2 col[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) col[n1] = a[n1][k2];
    Dft<A, DIR>::run(col);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) a[k1][k2] = col[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[(k1 * B * tB + k2 * A * tA) % N] = a[k1][k2];
}

template <int DIR>
struct Dft<6, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<2, 3, DIR>(v); }
};
template <int DIR>
struct Dft<12, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<4, 3, DIR>(v); }
};
template <int DIR>
struct Dft<24, DIR> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<8, 3, DIR>(v); }
};

// ---- stages --------------------------------------------------------------------

// positions are unsigned: divisions by the constant spans then need no sign fix-ups
template <int N, int T, int R, int NS>
__device__ __forceinline__ int out_pos(int tl, int c, int r) {
  const unsigned j = unsigned(tl) + unsigned(T * c);
  return int((j / unsigned(NS)) * unsigned(NS * R) + (j % unsigned(NS)) + unsigned(r * NS));
}
template <int N, int T, int R>
__device__ __forceinline__ int in_pos(int tl, int c, int r) {
  return tl + T * c + r * (N / R);
}

// twiddle + DFT of every butterfly of one stage (tw[t] = exp(-2 pi i t / N))
template <int N, int T, int DIR, int R, int NS>
__device__ __forceinline__ void stage(double2* v, int tl, const double2* __restrict__ tw) {
  constexpr int E = N / T;
  constexpr int NB = E / R;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (NS > 1) {
      const int jm = (tl + T * c) % NS;
      const int step = jm * (N / (NS * R));
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[r * step];
        if (DIR > 0) w.y = -w.y;
        v[c * R + r] = cmul(v[c * R + r], w);
      }
    }
    Dft<R, DIR>::run(v + c * R);
  }
}

// LDS addressing of position p of the line owned by this thread group: PADDIV > 0 inserts one pad slot
// every PADDIV positions; PADDIV = -(100 K + M) permutes positions within aligned blocks instead,
// p ^ ((p >> K) & M), which spreads strided accesses over the banks at no extra LDS and with a shift,
// a mask and an exclusive or per address (no division)
template <int PADDIV>
__device__ __forceinline__ int padded(int p) {
  if constexpr (PADDIV < 0) {
    constexpr unsigned K = unsigned(-PADDIV) / 100u, M = unsigned(-PADDIV) % 100u;
    return int(unsigned(p) ^ ((unsigned(p) >> K) & M));
  } else {
    return PADDIV > 0 ? int(unsigned(p) + unsigned(p) / unsigned(PADDIV)) : p;
  }
}

// Move stage outputs (radix Ra, span NSa) to the next stage's inputs (radix Rb)
// through LDS, real then imaginary part.  `base` is this line's LDS offset.
template <int N, int T, int Ra, int NSa, int Rb, int PADDIV>
__device__ __forceinline__ void exchange(double2* v, double* lds, int base, int tl) {
  constexpr int E = N / T;
  double tmp[E];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E / Ra; ++c)
#pragma unroll
    for (int r = 0; r < Ra; ++r) lds[base + padded<PADDIV>(out_pos<N, T, Ra, NSa>(tl, c, r))] = v[c * Ra + r].x;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E / Rb; ++c)
#pragma unroll
    for (int r = 0; r < Rb; ++r) tmp[c * Rb + r] = lds[base + padded<PADDIV>(in_pos<N, T, Rb>(tl, c, r))];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E / Ra; ++c)
#pragma unroll
    for (int r = 0; r < Ra; ++r) lds[base + padded<PADDIV>(out_pos<N, T, Ra, NSa>(tl, c, r))] = v[c * Ra + r].y;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < E / Rb; ++c)
#pragma unroll
    for (int r = 0; r < Rb; ++r) {
      const int k = c * Rb + r;
      v[k] = make_double2(tmp[k], lds[base + padded<PADDIV>(in_pos<N, T, Rb>(tl, c, r))]);
    }
}

// Ordering point between LDS writes and reads of one wavefront.  LDS
// operations of a wave are performed in issue order, so threads of one wave
// exchanging through LDS need only keep the compiler from reordering.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ordering for a line of T consecutive threads: wave-level when every line
// lies within one wavefront (T divides 64), else a block barrier.
template <int T>
__device__ __forceinline__ void line_sync() {
  if constexpr (64 % T == 0) wave_sync();
  else __syncthreads();
}

// Exchange for lines of T consecutive threads: complex values.
template <int N, int T, int Ra, int NSa, int Rb, int PADDIV>
__device__ __forceinline__ void exchange_wave(double2* v, double2* lds, int base, int tl) {
  constexpr int E = N / T;
  line_sync<T>();
#pragma unroll
  for (int c = 0; c < E / Ra; ++c)
#pragma unroll
    for (int r = 0; r < Ra; ++r) lds[base + padded<PADDIV>(out_pos<N, T, Ra, NSa>(tl, c, r))] = v[c * Ra + r];
  line_sync<T>();
#pragma unroll
  for (int c = 0; c < E / Rb; ++c)
#pragma unroll
    for (int r = 0; r < Rb; ++r) v[c * Rb + r] = lds[base + padded<PADDIV>(in_pos<N, T, Rb>(tl, c, r))];
}

template <int N, int T, int DIR, int R0, int R1, int R2, int R3, int PADDIV>
__device__ __forceinline__ void run_wave(double2* v, double2* lds, int base, int tl, const double2* __restrict__ tw) {
  static_assert(R0 * R1 * R2 * R3 == N, "radices must multiply to N");
  constexpr int NS1 = R0, NS2 = R0 * R1, NS3 = R0 * R1 * R2;
  stage<N, T, DIR, R0, 1>(v, tl, tw);
  if constexpr (R1 > 1) {
    exchange_wave<N, T, R0, 1, R1, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R1, NS1>(v, tl, tw);
  }
  if constexpr (R2 > 1) {
    exchange_wave<N, T, R1, NS1, R2, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R2, NS2>(v, tl, tw);
  }
  if constexpr (R3 > 1) {
    exchange_wave<N, T, R2, NS2, R3, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R3, NS3>(v, tl, tw);
  }
}

// Full transform.  Ends with the last stage's outputs in registers; the
// caller must not write `lds` before a __syncthreads().
template <int N, int T, int DIR, int R0, int R1, int R2, int R3, int PADDIV>
__device__ __forceinline__ void run(double2* v, double* lds, int base, int tl, const double2* __restrict__ tw) {
  static_assert(R0 * R1 * R2 * R3 == N, "radices must multiply to N");
  static_assert(R0 == N / T, "stage 0 takes one butterfly per thread: v[r] = x[tl + T r] are its inputs");
  static_assert((N / T) % R0 == 0 && (N / T) % R1 == 0 && (N / T) % R2 == 0 && (N / T) % R3 == 0,
                "every radix must divide N/T");
  constexpr int NS1 = R0, NS2 = R0 * R1, NS3 = R0 * R1 * R2;
  stage<N, T, DIR, R0, 1>(v, tl, tw);
  if constexpr (R1 > 1) {
    exchange<N, T, R0, 1, R1, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R1, NS1>(v, tl, tw);
  }
  if constexpr (R2 > 1) {
    exchange<N, T, R1, NS1, R2, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R2, NS2>(v, tl, tw);
  }
  if constexpr (R3 > 1) {
    exchange<N, T, R2, NS2, R3, PADDIV>(v, lds, base, tl);
    stage<N, T, DIR, R3, NS3>(v, tl, tw);
  }
}

// ---- lines of one wavefront (or less) with LDS twiddles ------------------------
//
// Variant for kernels whose LDS budget is tight: the exchange moves real and
// imaginary planes of doubles one after the other, and the stage twiddles come
// from LDS tables, one per stage s >= 1, of NS_s entries
// tws[m] = exp(-2 pi i m / (NS_s R_s)), so that the lanes of a wave read
// consecutive entries.  Only the first power w of a butterfly is read; w^r
// follows by repeated products (rounding grows like r ulp, far below the
// transform's own error).

template <int R0, int R1, int R2, int R3>
struct StageTw {
  static constexpr int NS1 = R0, NS2 = R0 * R1, NS3 = R0 * R1 * R2;
  static constexpr int OFF1 = 0, OFF2 = (R1 > 1 ? NS1 : 0), OFF3 = OFF2 + (R2 > 1 ? NS2 : 0);
  static constexpr int SIZE = OFF3 + (R3 > 1 ? NS3 : 0);
};

// fill the stage tables from tw[t] = exp(-2 pi i t / N), t < N/2
template <int N, int R0, int R1, int R2, int R3>
__device__ __forceinline__ void fill_stage_tw(double2* twl, const double2* __restrict__ tw, int tid, int nthreads) {
  using ST = StageTw<R0, R1, R2, R3>;
  for (int t = tid; t < ST::SIZE; t += nthreads) {
    int m, step;
    if (t < ST::OFF2 || (R2 == 1 && R3 == 1)) {
      m = t - ST::OFF1;
      step = N / (ST::NS1 * R1);
    } else if (t < ST::OFF3 || R3 == 1) {
      m = t - ST::OFF2;
      step = N / (ST::NS2 * R2);
    } else {
      m = t - ST::OFF3;
      step = N / (ST::NS3 * (R3 > 1 ? R3 : 1));
    }
    twl[t] = tw[m * step];
  }
}

template <int N, int T, int DIR, int R, int NS>
__device__ __forceinline__ void stage_lt(double2* v, int tl, const double2* tws) {
  constexpr int E = N / T;
  constexpr int NB = E / R;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if constexpr (NS > 1) {
      const int jm = int((unsigned(tl) + unsigned(T * c)) % unsigned(NS));
      double2 w1 = tws[jm];
      if (DIR > 0) w1.y = -w1.y;
      double2 w = w1;
      v[c * R + 1] = cmul(v[c * R + 1], w1);
#pragma unroll
      for (int r = 2; r < R; ++r) {
        w = cmul(w, w1);
        v[c * R + r] = cmul(v[c * R + r], w);
      }
    }
    Dft<R, DIR>::run(v + c * R);
  }
}

// BLK: the T threads of a line are spread over the block (not consecutive
// lanes), so every ordering point is a block barrier.
template <bool BLK, int T>
__device__ __forceinline__ void xsync() {
  if constexpr (BLK) __syncthreads();
  else line_sync<T>();
}

template <int N, int T, int Ra, int NSa, int Rb, int PADDIV, bool BLK = false>
__device__ __forceinline__ void exchange_split(double2* v, double* lds, int base, int tl) {
  constexpr int E = N / T;
  double tmp[E];
  xsync<BLK, T>();
#pragma unroll
  for (int c = 0; c < E / Ra; ++c)
#pragma unroll
    for (int r = 0; r < Ra; ++r) lds[base + padded<PADDIV>(out_pos<N, T, Ra, NSa>(tl, c, r))] = v[c * Ra + r].x;
  xsync<BLK, T>();
#pragma unroll
  for (int c = 0; c < E / Rb; ++c)
#pragma unroll
    for (int r = 0; r < Rb; ++r) tmp[c * Rb + r] = lds[base + padded<PADDIV>(in_pos<N, T, Rb>(tl, c, r))];
  xsync<BLK, T>();
#pragma unroll
  for (int c = 0; c < E / Ra; ++c)
#pragma unroll
    for (int r = 0; r < Ra; ++r) lds[base + padded<PADDIV>(out_pos<N, T, Ra, NSa>(tl, c, r))] = v[c * Ra + r].y;
  xsync<BLK, T>();
#pragma unroll
  for (int c = 0; c < E / Rb; ++c)
#pragma unroll
    for (int r = 0; r < Rb; ++r) {
      const int k = c * Rb + r;
      v[k] = make_double2(tmp[k], lds[base + padded<PADDIV>(in_pos<N, T, Rb>(tl, c, r))]);
    }
}

template <int N, int T, int DIR, int R0, int R1, int R2, int R3, int PADDIV, bool BLK = false>
__device__ __forceinline__ void run_split(double2* v, double* lds, int base, int tl, const double2* twl) {
  static_assert(R0 * R1 * R2 * R3 == N, "radices must multiply to N");
  static_assert(R0 == N / T, "stage 0 takes one butterfly per thread: v[r] = x[tl + T r] are its inputs");
  static_assert((N / T) % R0 == 0 && (N / T) % R1 == 0 && (N / T) % R2 == 0 && (N / T) % R3 == 0,
                "every radix must divide N/T");
  using ST = StageTw<R0, R1, R2, R3>;
  stage_lt<N, T, DIR, R0, 1>(v, tl, twl);
  if constexpr (R1 > 1) {
    exchange_split<N, T, R0, 1, R1, PADDIV, BLK>(v, lds, base, tl);
    stage_lt<N, T, DIR, R1, ST::NS1>(v, tl, twl + ST::OFF1);
  }
  if constexpr (R2 > 1) {
    exchange_split<N, T, R1, ST::NS1, R2, PADDIV, BLK>(v, lds, base, tl);
    stage_lt<N, T, DIR, R2, ST::NS2>(v, tl, twl + ST::OFF2);
  }
  if constexpr (R3 > 1) {
    exchange_split<N, T, R2, ST::NS2, R3, PADDIV, BLK>(v, lds, base, tl);
    stage_lt<N, T, DIR, R3, ST::NS3>(v, tl, twl + ST::OFF3);
  }
}

// radix of the last stage
template <int R0, int R1, int R2, int R3>
struct Last {
  static constexpr int value = R3 > 1 ? R3 : (R2 > 1 ? R2 : (R1 > 1 ? R1 : R0));
};

}  // namespace rf
}  // namespace lmvd
