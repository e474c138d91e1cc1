// Batched complex FFTs of one workgroup over lines held in LDS.
//
// Mixed-radix (2, 3, 4, 8) Stockham autosort passes, in place: every pass
// loads its butterflies' inputs into registers (twiddled on load), waits at a
// barrier, and writes the butterfly outputs back in natural-order position.
// Twiddles come from a host table tw[t] = exp(-2 pi i t / n), t < n.
// DIR = -1 computes sum_t x_t e^{-2 pi i k t/n}, DIR = +1 the same with e^{+...};
// neither is normalised.
#pragma once

#include <hip/hip_runtime.h>

namespace lmvd {

constexpr int kMaxStagesDev = 12;

struct FftDev {
  int n;
  int nstages;
  int radix[kMaxStagesDev];
  int ns[kMaxStagesDev];
  const double2* tw;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// (S i) z for S = +1 or -1
template <int S>
__device__ __forceinline__ double2 mul_si(double2 z) {
  return (S > 0) ? make_double2(-z.y, z.x) : make_double2(z.y, -z.x);
}

template <int R, int DIR>
__device__ __forceinline__ void small_dft(double2* v);

template <>
__device__ __forceinline__ void small_dft<1, -1>(double2*) {}
template <>
__device__ __forceinline__ void small_dft<1, 1>(double2*) {}

template <>
__device__ __forceinline__ void small_dft<2, -1>(double2* v) {
  double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <>
__device__ __forceinline__ void small_dft<2, 1>(double2* v) {
  small_dft<2, -1>(v);
}

// 3-point: X1,2 = a - (b+c)/2 +- DIR i (sqrt 3 / 2)(b - c)
template <int DIR>
__device__ __forceinline__ void dft3(double2* v) {
  const double h3 = 0.86602540378443864676;  // sqrt(3)/2
  double2 a = v[0], b = v[1], c = v[2];
  double2 t1 = cadd(b, c);
  double2 t2 = make_double2(a.x - 0.5 * t1.x, a.y - 0.5 * t1.y);
  double2 t3 = cscale(csub(b, c), h3);
  v[0] = cadd(a, t1);
  v[1] = cadd(t2, mul_si<DIR>(t3));
  v[2] = csub(t2, mul_si<DIR>(t3));
}
template <>
__device__ __forceinline__ void small_dft<3, -1>(double2* v) { dft3<-1>(v); }
template <>
__device__ __forceinline__ void small_dft<3, 1>(double2* v) { dft3<1>(v); }

template <int DIR>
__device__ __forceinline__ void dft4(double2& a, double2& b, double2& c, double2& d) {
  double2 s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = csub(b, d);
  a = cadd(s0, s2);
  c = csub(s0, s2);
  b = cadd(s1, mul_si<DIR>(s3));
  d = csub(s1, mul_si<DIR>(s3));
}
template <>
__device__ __forceinline__ void small_dft<4, -1>(double2* v) { dft4<-1>(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void small_dft<4, 1>(double2* v) { dft4<1>(v[0], v[1], v[2], v[3]); }

// 8-point as two 4-point DFTs of the even and odd samples
template <int DIR>
__device__ __forceinline__ void dft8(double2* v) {
  const double r2 = 0.70710678118654752440;  // sqrt(2)/2
  double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // W8^k = exp(DIR 2 pi i k / 8)
  double2 w1o = make_double2(r2 * (o1.x - DIR * o1.y), r2 * (o1.y + DIR * o1.x));  // (1 + DIR i) r2 * o1
  double2 w2o = mul_si<DIR>(o2);
  double2 w3o = make_double2(r2 * (-o3.x - DIR * o3.y), r2 * (-o3.y + DIR * o3.x));  // (-1 + DIR i) r2 * o3
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1o);
  v[5] = csub(e1, w1o);
  v[2] = cadd(e2, w2o);
  v[6] = csub(e2, w2o);
  v[3] = cadd(e3, w3o);
  v[7] = csub(e3, w3o);
}
template <>
__device__ __forceinline__ void small_dft<8, -1>(double2* v) { dft8<-1>(v); }
template <>
__device__ __forceinline__ void small_dft<8, 1>(double2* v) { dft8<1>(v); }

// One Stockham pass of radix R over `nlines` lines of length n (stride ld).
// MAXE bounds the elements a thread stages: nlines * n <= MAXE * nth.
template <int R, int DIR, int MAXE>
__device__ __forceinline__ void fft_pass(double2* buf, int ld, int nlines, int n, int Ns,
                                         const double2* __restrict__ tw, int tid, int nth) {
  constexpr int MAXBF = (MAXE + R - 1) / R;
  const int nbf = n / R;
  const int total = nbf * nlines;
  const int tws = n / (Ns * R);
  double2 v[MAXBF][R];
  int dst[MAXBF];
#pragma unroll
  for (int it = 0; it < MAXBF; ++it) {
    const int b = tid + it * nth;
    dst[it] = -1;
    if (b < total) {
      const int line = b / nbf;
      const int j = b - line * nbf;
      const int jm = j % Ns;
      const double2* x = buf + line * ld;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 val = x[j + r * nbf];
        if (r > 0 && jm > 0) {
          double2 w = tw[r * jm * tws];
          if (DIR > 0) w.y = -w.y;
          val = cmul(val, w);
        }
        v[it][r] = val;
      }
      dst[it] = line * ld + (j / Ns) * Ns * R + jm;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXBF; ++it) {
    if (dst[it] >= 0) {
      small_dft<R, DIR>(v[it]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[it] + r * Ns] = v[it][r];
    }
  }
  __syncthreads();
}

// Full transform of `nlines` lines in LDS.  Caller must __syncthreads() after
// filling the buffer; the function ends with a barrier.
template <int DIR, int MAXE>
__device__ void fft_lines(double2* buf, int ld, int nlines, const FftDev& f, int tid, int nth) {
  for (int s = 0; s < f.nstages; ++s) {
    switch (f.radix[s]) {
      case 8: fft_pass<8, DIR, MAXE>(buf, ld, nlines, f.n, f.ns[s], f.tw, tid, nth); break;
      case 4: fft_pass<4, DIR, MAXE>(buf, ld, nlines, f.n, f.ns[s], f.tw, tid, nth); break;
      case 3: fft_pass<3, DIR, MAXE>(buf, ld, nlines, f.n, f.ns[s], f.tw, tid, nth); break;
      case 2: fft_pass<2, DIR, MAXE>(buf, ld, nlines, f.n, f.ns[s], f.tw, tid, nth); break;
      default: break;
    }
  }
}

}  // namespace lmvd
