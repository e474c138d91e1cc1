// MI355X (gfx950) implementation of one explicit RK2 substep of the
// low-Mach variable-density pseudospectral method (Algorithm
// time_advanceDNS of Reuter, Oliver & Moser), behind the C ABI of lmvd.h.
//
// Data never leaves the plane-major spectral layout [j][n_idx][l]:
//  * "column" work (banded y-operations per wavenumber pair) runs one thread
//    per (l, n) column and sweeps j; neighbouring threads touch neighbouring
//    l, so every access of a sweep is coalesced and no transpose is needed;
//  * "plane" work (3/2-rule transforms and pointwise products) runs per
//    y-plane in three kernels: evaluation at the Greville point + inverse
//    z-FFT (k_eval_zinv), inverse x-FFT + products + forward x-FFT
//    (k_xpass), forward z-FFT + truncation (k_zfwd).  Physical fields exist
//    only in registers inside k_xpass.
// Everything is float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lmvd.h"
#include "fft_lds.h"
#include "fft_reg.h"
#include "plan_host.h"

namespace lmvd {

constexpr int kMaxIn = 8;
constexpr int kMaxOut = 10;
constexpr int kNumAux = 4;   // physical-grid fields fixed during a substep
// The column sweeps run one thread per column, a dependent chain of row steps each; at two waves per
// SIMD they hide the HBM latency only with their loads issued well ahead of use. A regular stream (one
// row per step of its sweep) is read through a ring whose slot d serves the steps d (mod depth): the
// sweep runs in blocks of `depth` steps, unrolled, and each step consumes its slot, then refills it with
// an unconditional load (row index clamped into range); consuming before the load is issued lets the
// load take the slot's register. A ring that shifts its entries instead (slot 0 consumed, slot d+1
// copied to slot d) copies each load's destination one step after issuing it, and the copy waits for
// the load, so such a ring hides one step of latency at most. Depths: the m^c sweeps read kPreMc
// (sweep 1), kPreMc2 (sweep 2) and kPreMc3 (sweep 3, rows and factor rows) steps ahead, the transposed
// A(k) solve kFacPre.
constexpr int kPreMc = 8, kFacPre = 3, kPreMc2 = 4, kPreMc3 = 4;
constexpr int kThreads = 256;
constexpr int kZMaxE = 12;    // elements per thread in the z-FFT kernels
constexpr int kXSlots = 3;    // complex slots per thread per line set in k_xpass
constexpr int kNumEv = 4;     // E0, E1, E2 (B at tau), F0 (B* at tau)

enum EvalKind { EV_E0 = 0, EV_E1 = 1, EV_E2 = 2, EV_F0 = 3, EV_LAP = 4, EV_IDENT = 5 };
enum Mult { MU_ONE = 0, MU_IK1 = 1, MU_IK3 = 2, MU_K1K = 3, MU_K3K = 4 };
// PH_RZV: R_z with rho D = rho D(z); PH_TAU: tau_ij = mu(z) S_ij (variable transport laws)
enum Phase { PH_RZ = 0, PH_RHOT = 1, PH_L = 2, PH_VEL = 3, PH_TOPHYS = 5, PH_FROMPHYS = 6, PH_RZV = 7, PH_TAU = 8 };
enum Epi { EPI_STORE = 0, EPI_ADD = 1, EPI_ADD_ZUPDATE = 2 };

// Read-only plan tables live in the constant address space: the kernels read
// them with indices that are uniform across a wavefront (row numbers), which
// lets the compiler use scalar loads for them.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
inline cptr<T> to_cptr(const void* p) { return (cptr<T>)(p); }

struct DevPlan {
  int n2, p, nl, nn, n3, m1, m3, hx;
  double dt, mu, rhoD, g, rho_l, rho_h, inv_rlrh, drho;
  // row tables
  cptr<int> ev_lo;        // [kNumEv][n2]
  cptr<double> ev_w;      // [kNumEv][n2][kMaxW]
  cptr<int> gs_lo;        // [2][n2+1]   G0, G1 at tau*
  cptr<double> gs_w;
  cptr<int> es_lo;        // [3][n2+1]   E*_0, E*_1, E*_2 at tau*
  cptr<double> es_w;
  cptr<double> dstar;     // [n2]
  cptr<double> lu_l;      // [3][n2][kMaxBand]
  cptr<double> lu_u;      // [3][n2][kMaxBand+1]
  cptr<double> lu_uinv;   // [3][n2]
  cptr<double> lu_ut;     // [3][n2][kMaxBand+1] row i: U_{i-1-q, i} (q < kMaxBand, 0 above row 0), then 1/U_ii
  cptr<double> lu_lt;     // [3][n2][kMaxBand]   row i: L_{i+1+m, i} (0 below the last row)
  const double* k1;        // [nl]
  const double* k3;        // [nn]
  cptr<int> emit_first;   // [n2] first E0 row whose band starts at row i
  cptr<int> emit_cnt;     // [n2] number of such rows
  cptr<int> g1e_cnt;      // [n2] interior tau* rows whose G1 band starts at B row j (emitted in descending row order)
  cptr<int> asc_first;    // [n2+1] first tau row whose last F0/F1 column is B* row j
  cptr<int> asc_cnt;      // [n2+1]
  cptr<double> asc_w;     // [2][n2][kMaxW] F0, F1 weights of c_{last - q}
  const double* fac;       // bottom-up factors of A(k) per (l, |n|) pair: row i at slot fac_off[i], [slots][npairs]
  cptr<int> fac_nm;       // [n2+1] multipliers of row i (rows i+1 .. i+nm)
  cptr<int> fac_ns;       // [n2+1] entries of row i left of its diagonal
  cptr<int> fac_off;      // [n2+1] first slot of row i
  // by columns, for the transposed A(k) solve (slot -1: no entry): step i of L^T w = b reads the left
  // entry q of row i+1+q (q < kFacMax) and then the inverse pivot of row i; step i of U^T psi = w reads
  // multiplier m of row i-1-m
  cptr<int> fac_lt;       // [n2+1][kFacMax+1]
  cptr<int> fac_ut;       // [n2+1][kFacMax]
  FftDev fz, fx;
  const double2* xtw;      // [hx] exp(-2 pi i k / m1)
  cptr<double> wall_w;    // weights of the wall rows of E0 P_N (interior values -> wall values)
  int wall_k0, wall_k1;   // interior planes entering the lower / upper wall value
  // transport laws (Section 2): mu(z) = mu + mu_z . (z, z^2, z^3); q(z) = rhoD + rq_z . (z, z^2, z^3);
  // rho D_z = q(z) (rq_form 0) or f(z) q(z) (rq_form 1)
  double mu_z[3], rq_z[3];
  int rq_form;
};

struct EvalIn {
  const double2* a;
  const double2* b;
  int kind;
  int ma;
  int mb;
  int slot;  // zbuf slot the inverse z transform writes (-1 before plane_phase: the input's position)
};
struct EvalArgs {
  EvalIn in[kMaxIn];
};
struct OutPtrs {
  double2* v[kMaxOut];
};

// ---------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 fma2(double s, double2 a, double2 acc) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}
__device__ __forceinline__ double2 times_i(double2 z) { return make_double2(-z.y, z.x); }

// transport laws at a physical point: mu(z), and rho D_z with its z-derivative (rho = f(z) given)
__device__ __forceinline__ double mu_of(const DevPlan& P, double z) {
  return fma(fma(fma(P.mu_z[2], z, P.mu_z[1]), z, P.mu_z[0]), z, P.mu);
}
__device__ __forceinline__ void rhod_of(const DevPlan& P, double z, double rho, double& k, double& dk) {
  const double q = fma(fma(fma(P.rq_z[2], z, P.rq_z[1]), z, P.rq_z[0]), z, P.rhoD);
  const double dq = fma(fma(3.0 * P.rq_z[2], z, 2.0 * P.rq_z[1]), z, P.rq_z[0]);
  if (P.rq_form == 0) {
    k = q;
    dk = dq;
  } else {  // f'(z) = rho^2 (rh - rl) / (rl rh)
    k = rho * q;
    dk = fma(rho * rho * P.drho * P.inv_rlrh, q, rho * dq);
  }
}

// spectral multiplier of a column
__device__ __forceinline__ double2 apply_mult(int m, double k1, double k3, double2 v) {
  switch (m) {
    case MU_IK1: return make_double2(-k1 * v.y, k1 * v.x);
    case MU_IK3: return make_double2(-k3 * v.y, k3 * v.x);
    case MU_K1K:
    case MU_K3K: {
      double ksq = k1 * k1 + k3 * k3;
      if (ksq == 0.0) return zero2();
      double s = ((m == MU_K1K) ? k1 : k3) / sqrt(ksq);
      return cscale(v, s);
    }
    default: return v;
  }
}

// value at tau_j of column (ni, l) of a spectral coefficient array
__device__ __forceinline__ double2 eval_at(const DevPlan& P, int kind, const double2* __restrict__ src,
                                           int j, size_t col, size_t ncol, double ksq) {
  if (kind == EV_IDENT) return src[size_t(j) * ncol + col];
  const int rows = (kind == EV_F0) ? P.n2 + 1 : P.n2;
  const int kk = (kind == EV_LAP) ? EV_E2 : kind;
  const int lo = P.ev_lo[kk * P.n2 + j];
  const auto w = P.ev_w + (size_t(kk) * P.n2 + j) * kMaxW;
  const auto w0 = P.ev_w + (size_t(EV_E0) * P.n2 + j) * kMaxW;
  double2 acc = zero2(), acc0 = zero2();
#pragma unroll
  for (int q = 0; q < kMaxW; ++q) {
    const int r = lo + q;
    if (r < rows && (w[q] != 0.0 || (kind == EV_LAP && w0[q] != 0.0))) {
      const double2 s = src[size_t(r) * ncol + col];
      acc = fma2(w[q], s, acc);
      if (kind == EV_LAP) acc0 = fma2(w0[q], s, acc0);
    }
  }
  if (kind == EV_LAP) acc = make_double2(acc.x - ksq * acc0.x, acc.y - ksq * acc0.y);
  return acc;
}

// ---------------------------------------------------------------------------
// plane kernel 1: evaluation at tau_j, spectral multiplier, inverse z-FFT
// grid (ceil(nl/LG), planes, nin); output zbuf[f][jj][b][l]

__global__ void __launch_bounds__(kThreads) k_eval_zinv(DevPlan P, EvalArgs A, double2* __restrict__ zbuf,
                                                        int j0, int pb, int LG) {
  extern __shared__ double2 lds[];
  const int f = blockIdx.z, jj = blockIdx.y, j = j0 + jj, l0 = blockIdx.x * LG;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int M3 = P.m3, nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = M3 - nn;
  const EvalIn in = A.in[f];
  const size_t ncol = size_t(nn) * nl;
  // zero the padded (dealiasing) positions
  for (int idx = tid; idx < LG * pad; idx += nth) {
    const int ll = idx % LG, q = idx / LG;
    lds[ll * M3 + h3 + q] = zero2();
  }
  // retained modes
  for (int idx = tid; idx < LG * nn; idx += nth) {
    const int ll = idx % LG, ni = idx / LG, l = l0 + ll;
    double2 v = zero2();
    if (l < nl) {
      const double k1 = P.k1[l], k3 = P.k3[ni];
      const double ksq = k1 * k1 + k3 * k3;
      const size_t col = size_t(ni) * nl + l;
      v = apply_mult(in.ma, k1, k3, eval_at(P, in.kind, in.a, j, col, ncol, ksq));
      if (in.b) {
        const double2 w = apply_mult(in.mb, k1, k3, eval_at(P, in.kind, in.b, j, col, ncol, ksq));
        v = cadd(v, w);
      }
    }
    const int pos = (ni < h3) ? ni : ni + pad;
    lds[ll * M3 + pos] = v;
  }
  __syncthreads();
  fft_lines<1, kZMaxE>(lds, M3, LG, P.fz, tid, nth);
  double2* out = zbuf + (size_t(A.in[f].slot) * pb + jj) * size_t(M3) * nl;
  for (int idx = tid; idx < LG * M3; idx += nth) {
    const int ll = idx % LG, b = idx / LG;
    if (l0 + ll < nl) out[size_t(b) * nl + l0 + ll] = lds[ll * M3 + b];
  }
}

// ---------------------------------------------------------------------------
// pointwise products on the physical grid

template <int PH>
struct Op;

// Fields fixed during a substep live on the physical grid (aux, field stride
// fs): g_i = -(1/rho) d_i z (i = 1..3) and f'(z) = rho^2 (rh - rl)/(rl rh),
// written by the R_z phase and read by every L and rho_t phase.
template <>
struct Op<PH_RZ> {  // R_z = (1/rho)(-m^d . grad z + rho D lap z); inputs lap z, z, z1, m1, z2, m2, z3, m3
  static constexpr int NIN = 8, NOUT = 1;
  __device__ static void apply(const DevPlan& P, const double* x, double* y, double* a, size_t fs) {
    const double ir = (P.rho_h - P.drho * x[1]) * P.inv_rlrh;
    const double rho = (P.rho_l * P.rho_h) / (P.rho_h - P.drho * x[1]);
    a[0] = -ir * x[2];
    a[fs] = -ir * x[4];
    a[2 * fs] = -ir * x[6];
    a[3 * fs] = rho * rho * P.drho * P.inv_rlrh;
    y[0] = (P.rhoD * x[0] - (x[2] * x[3] + x[4] * x[5] + x[6] * x[7])) * ir;
  }
};
template <>
struct Op<PH_RZV> {  // R_z = (1/rho)(-m^d . grad z + rho D(z) lap z + (rho D)'(z) |grad z|^2); inputs as PH_RZ
  static constexpr int NIN = 8, NOUT = 1;
  __device__ static void apply(const DevPlan& P, const double* x, double* y, double* a, size_t fs) {
    const double ir = (P.rho_h - P.drho * x[1]) * P.inv_rlrh;
    const double rho = (P.rho_l * P.rho_h) / (P.rho_h - P.drho * x[1]);
    double k, dk;
    rhod_of(P, x[1], rho, k, dk);
    a[0] = -ir * x[2];
    a[fs] = -ir * x[4];
    a[2 * fs] = -ir * x[6];
    a[3 * fs] = rho * rho * P.drho * P.inv_rlrh;
    const double g2 = x[2] * x[2] + x[4] * x[4] + x[6] * x[6];
    y[0] = (k * x[0] + dk * g2 - (x[2] * x[3] + x[4] * x[5] + x[6] * x[7])) * ir;
  }
};
template <>
struct Op<PH_TAU> {  // tau = mu(z) S for three strain components; inputs S_a, S_b, S_c, z
  static constexpr int NIN = 4, NOUT = 3;
  __device__ static void apply(const DevPlan& P, const double* x, double* y, double*, size_t) {
    const double mu = mu_of(P, x[3]);
#pragma unroll
    for (int q = 0; q < 3; ++q) y[q] = mu * x[q];
  }
};
template <>
struct Op<PH_RHOT> {  // rho_t = f'(z) z_t; input z_t
  static constexpr int NIN = 1, NOUT = 1;
  __device__ static void apply(const DevPlan&, const double* x, double* y, double* a, size_t fs) {
    y[0] = a[3 * fs] * x[0];
  }
};
template <>
struct Op<PH_L> {  // L z_t = -(1/rho) grad z . m^c = g . m^c; inputs m1c, m2c, m3c
  static constexpr int NIN = 3, NOUT = 1;
  __device__ static void apply(const DevPlan&, const double* x, double* y, double* a, size_t fs) {
    y[0] = a[0] * x[0] + a[fs] * x[1] + a[2 * fs] * x[2];
  }
};
template <>
struct Op<PH_VEL> {  // u = m / rho, rho, and C_ij = -m_i m_j / rho (i <= j)
  static constexpr int NIN = 4, NOUT = 10;
  __device__ static void apply(const DevPlan& P, const double* x, double* y, double*, size_t) {
    const double den = P.rho_h - P.drho * x[0];
    const double ir = den * P.inv_rlrh;
    const double u1 = x[1] * ir, u2 = x[2] * ir, u3 = x[3] * ir;
    y[0] = u1;
    y[1] = u2;
    y[2] = u3;
    y[3] = (P.rho_l * P.rho_h) / den;
    y[4] = -x[1] * u1;
    y[5] = -x[1] * u2;
    y[6] = -x[1] * u3;
    y[7] = -x[2] * u2;
    y[8] = -x[2] * u3;
    y[9] = -x[3] * u3;
  }
};
template <>
struct Op<PH_TOPHYS> {
  static constexpr int NIN = 1, NOUT = 0;
  __device__ static void apply(const DevPlan&, const double*, double*, double*, size_t) {}
};
template <>
struct Op<PH_FROMPHYS> {
  static constexpr int NIN = 0, NOUT = 1;
  __device__ static void apply(const DevPlan&, const double*, double*, double*, size_t) {}
};

// ---------------------------------------------------------------------------
// plane kernel 2: per (plane, group of z lines): inverse real x-FFT of every
// input (length m1 via a complex FFT of m1/2), products, forward real x-FFT
// of every output.  grid (ceil(m3/BG), planes).

template <int PH>
__global__ void __launch_bounds__(kThreads) k_xpass(DevPlan P, const double2* __restrict__ zbuf,
                                                    double2* __restrict__ obuf, int pb, int BG,
                                                    double* phys_out, const double* phys_in, int j0,
                                                    double* __restrict__ aux) {
  using O = Op<PH>;
  constexpr int NIN = O::NIN, NOUT = O::NOUT;
  constexpr int NINA = NIN > 0 ? NIN : 1, NOUTA = NOUT > 0 ? NOUT : 1;
  extern __shared__ double2 lds[];
  const int jj = blockIdx.y, b0 = blockIdx.x * BG;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int H = P.hx, nl = P.nl, M3 = P.m3, M1 = P.m1;
  const int nlines = min(BG, M3 - b0);
  const int nel = nlines * H;
  double2 ph[NINA][kXSlots];
  double2 res[NOUTA][kXSlots];

#pragma unroll
  for (int f = 0; f < NIN; ++f) {
    const double2* X0 = zbuf + ((size_t(f) * pb + jj) * M3 + b0) * nl;
    for (int idx = tid; idx < nel; idx += nth) {
      const int line = idx / H, k = idx - line * H;
      const double2* X = X0 + size_t(line) * nl;
      const double2 a = (k < nl) ? X[k] : zero2();
      const double2 c = (k > 0 && H - k < nl) ? cconj(X[H - k]) : zero2();
      const double2 s = cadd(a, c), d = csub(a, c);
      const double2 w = cconj(P.xtw[k]);  // exp(+2 pi i k / m1)
      lds[idx] = cadd(s, times_i(cmul(w, d)));
    }
    __syncthreads();
    fft_lines<1, 6>(lds, H, nlines, P.fx, tid, nth);
#pragma unroll
    for (int s = 0; s < kXSlots; ++s) {
      const int idx = tid + s * nth;
      ph[f][s] = (idx < nel) ? lds[idx] : zero2();
    }
    if constexpr (PH == PH_TOPHYS) {
      double* dst = phys_out + (size_t(j0 + jj) * M3 + b0) * M1;
#pragma unroll
      for (int s = 0; s < kXSlots; ++s) {
        const int idx = tid + s * nth;
        if (idx < nel) {
          const int line = idx / H, m = idx - line * H;
          dst[size_t(line) * M1 + 2 * m] = ph[f][s].x;
          dst[size_t(line) * M1 + 2 * m + 1] = ph[f][s].y;
        }
      }
    }
    __syncthreads();
  }
  if constexpr (PH == PH_FROMPHYS) {
    const double* src = phys_in + (size_t(j0 + jj) * M3 + b0) * M1;
#pragma unroll
    for (int s = 0; s < kXSlots; ++s) {
      const int idx = tid + s * nth;
      if (idx < nel) {
        const int line = idx / H, m = idx - line * H;
        res[0][s] = make_double2(src[size_t(line) * M1 + 2 * m], src[size_t(line) * M1 + 2 * m + 1]);
      }
    }
  } else if constexpr (NOUT > 0) {
#pragma unroll
    for (int s = 0; s < kXSlots; ++s) {
      double xi[NINA], yo[NOUTA], xj[NINA], yp[NOUTA];
#pragma unroll
      for (int f = 0; f < NIN; ++f) {
        xi[f] = ph[f][s].x;
        xj[f] = ph[f][s].y;
      }
      const int idx = tid + s * nth;
      const int line = idx / H, m = idx - line * H;
      const size_t fs = size_t(P.n2) * M3 * M1;
      double* ap = aux ? aux + (size_t(j0 + jj) * M3 + b0 + (idx < nel ? line : 0)) * M1 + 2 * (idx < nel ? m : 0)
                       : nullptr;
      if (idx < nel) {
        O::apply(P, xi, yo, ap, fs);
        O::apply(P, xj, yp, ap ? ap + 1 : nullptr, fs);
      } else {
#pragma unroll
        for (int g = 0; g < NOUTA; ++g) yo[g] = yp[g] = 0.0;
      }
#pragma unroll
      for (int g = 0; g < NOUT; ++g) res[g][s] = make_double2(yo[g], yp[g]);
    }
  }
  const double scale = 1.0 / (double(M1) * double(M3));
#pragma unroll
  for (int g = 0; g < NOUT; ++g) {
#pragma unroll
    for (int s = 0; s < kXSlots; ++s) {
      const int idx = tid + s * nth;
      if (idx < nel) lds[idx] = res[g][s];
    }
    __syncthreads();
    fft_lines<-1, 6>(lds, H, nlines, P.fx, tid, nth);
    double2* Y0 = obuf + ((size_t(g) * pb + jj) * M3 + b0) * nl;
    for (int idx = tid; idx < nlines * nl; idx += nth) {
      const int line = idx / nl, l = idx - line * nl;
      const double2 Yk = lds[line * H + l];
      const double2 Yc = cconj(lds[line * H + ((H - l) % H)]);
      const double2 E = cscale(cadd(Yk, Yc), 0.5);
      const double2 D = csub(Yk, Yc);
      const double2 O = make_double2(0.5 * D.y, -0.5 * D.x);  // (Yk - conj Y_{H-k}) / (2i)
      const double2 Xt = cadd(E, cmul(P.xtw[l], O));
      Y0[size_t(line) * nl + l] = cscale(Xt, scale);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plane kernel 3: forward z-FFT, keep the retained n.  grid (ceil(nl/LG), planes, nout)

__global__ void __launch_bounds__(kThreads) k_zfwd(DevPlan P, const double2* __restrict__ obuf, OutPtrs V,
                                                   int j0, int pb, int LG) {
  extern __shared__ double2 lds[];
  const int g = blockIdx.z, jj = blockIdx.y, l0 = blockIdx.x * LG;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int M3 = P.m3, nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = M3 - nn;
  const double2* in = obuf + (size_t(g) * pb + jj) * size_t(M3) * nl;
  for (int idx = tid; idx < LG * M3; idx += nth) {
    const int ll = idx % LG, b = idx / LG;
    lds[ll * M3 + b] = (l0 + ll < nl) ? in[size_t(b) * nl + l0 + ll] : zero2();
  }
  __syncthreads();
  fft_lines<-1, kZMaxE>(lds, M3, LG, P.fz, tid, nth);
  double2* out = V.v[g] + size_t(j0 + jj) * nn * nl;
  for (int idx = tid; idx < LG * nn; idx += nth) {
    const int ll = idx % LG, ni = idx / LG;
    if (l0 + ll < nl) out[size_t(ni) * nl + l0 + ll] = lds[ll * M3 + ((ni < h3) ? ni : ni + pad)];
  }
}

// ---------------------------------------------------------------------------
// column kernels: values at the Greville points tau_j of spectral coefficient
// fields (one thread per (l, n) column, ascending sweep with a register
// window of coefficient rows, so every coefficient is read once).

struct RowWindow {
  double2 w[kMaxW];
  int base;
  __device__ __forceinline__ void init(const double2* __restrict__ src, size_t ncol, size_t c, int rows) {
    base = 0;
#pragma unroll
    for (int q = 0; q < kMaxW; ++q) w[q] = (q < rows) ? src[size_t(q) * ncol + c] : zero2();
  }
  __device__ __forceinline__ void advance(const double2* __restrict__ src, size_t ncol, size_t c, int rows, int lo) {
    while (base < lo) {
#pragma unroll
      for (int q = 0; q < kMaxW - 1; ++q) w[q] = w[q + 1];
      const int r = base + kMaxW;
      w[kMaxW - 1] = (r < rows) ? src[size_t(r) * ncol + c] : zero2();
      ++base;
    }
  }
  __device__ __forceinline__ double2 dot(cptr<double> wt) const {
    double2 acc = zero2();
#pragma unroll
    for (int q = 0; q < kMaxW; ++q) acc = fma2(wt[q], w[q], acc);
    return acc;
  }
};

// z -> E0 z, E1 z, (E2 - k^2 E0) z and i k3 E0 z at tau
struct ValuesZArgs {
  const double2* z;
  double2 *V0, *V1, *VL, *V3;
};
__device__ __forceinline__ void values_z_body(const DevPlan& P, size_t c, const ValuesZArgs& A) {
  const double2* __restrict__ z = A.z;
  double2* __restrict__ V0 = A.V0;
  double2* __restrict__ V1 = A.V1;
  double2* __restrict__ VL = A.VL;
  double2* __restrict__ V3 = A.V3;
  const size_t ncol = size_t(P.nn) * P.nl;
  if (c >= ncol) return;
  const int n2 = P.n2;
  const double k1 = P.k1[c % P.nl], k3 = P.k3[c / P.nl], ksq = k1 * k1 + k3 * k3;
  RowWindow rw;
  rw.init(z, ncol, c, n2);
  for (int i = 0; i < n2; ++i) {
    rw.advance(z, ncol, c, n2, P.ev_lo[i]);
    const double2 a0 = rw.dot(P.ev_w + size_t(i) * kMaxW);
    const double2 a1 = rw.dot(P.ev_w + (size_t(n2) + i) * kMaxW);
    const double2 a2 = rw.dot(P.ev_w + (size_t(2 * n2) + i) * kMaxW);
    const size_t e = size_t(i) * ncol + c;
    V0[e] = a0;
    V1[e] = a1;
    VL[e] = make_double2(a2.x - ksq * a0.x, a2.y - ksq * a0.y);
    V3[e] = times_i(cscale(a0, k3));
  }
}

// up to two B fields -> E0 values; one B* field -> F0 values (any pointer may be null)
__global__ void __launch_bounds__(kThreads) k_values(DevPlan P, const double2* __restrict__ a, double2* __restrict__ Va,
                                                     const double2* __restrict__ b, double2* __restrict__ Vb,
                                                     const double2* __restrict__ cs, double2* __restrict__ Vc) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int n2 = P.n2;
  RowWindow wa, wb, wc;
  if (a) wa.init(a, ncol, c, n2);
  if (b) wb.init(b, ncol, c, n2);
  if (cs) wc.init(cs, ncol, c, n2 + 1);
  for (int i = 0; i < n2; ++i) {
    const size_t e = size_t(i) * ncol + c;
    const auto w0 = P.ev_w + size_t(i) * kMaxW;
    if (a) {
      wa.advance(a, ncol, c, n2, P.ev_lo[i]);
      Va[e] = wa.dot(w0);
    }
    if (b) {
      wb.advance(b, ncol, c, n2, P.ev_lo[i]);
      Vb[e] = wb.dot(w0);
    }
    if (cs) {
      wc.advance(cs, ncol, c, n2 + 1, P.ev_lo[3 * n2 + i]);
      Vc[e] = wc.dot(P.ev_w + (size_t(3 * n2) + i) * kMaxW);
    }
  }
}

// BDF-like guess dt z_t^0 = a1 z + a2 h1 + a3 h2 + a4 h3 (eq. dzdt_guesses)
// (or zero) as coefficients, and its E0 values at tau
struct GuessArgs {
  const double2 *z, *h1, *h2, *h3;
  double a1, a2, a3, a4, dt;
  int zero;
  double2 *zt, *V;
};
__device__ __forceinline__ void guess_body(const DevPlan& P, size_t c, const GuessArgs& G) {
  const double2* __restrict__ z = G.z;
  const double2* __restrict__ h1 = G.h1;
  const double2* __restrict__ h2 = G.h2;
  const double2* __restrict__ h3 = G.h3;
  const double a1 = G.a1, a2 = G.a2, a3 = G.a3, a4 = G.a4, dt = G.dt;
  const int zero = G.zero;
  double2* __restrict__ zt = G.zt;
  double2* __restrict__ V = G.V;
  const size_t ncol = size_t(P.nn) * P.nl;
  if (c >= ncol) return;
  const int n2 = P.n2;
  auto coef = [&](int r) -> double2 {
    if (zero || r >= n2) return zero2();
    const size_t e = size_t(r) * ncol + c;
    const double2 A = z[e], B = h1[e], C = h2[e], D = h3[e];
    return make_double2((a1 * A.x + a2 * B.x + a3 * C.x + a4 * D.x) / dt,
                        (a1 * A.y + a2 * B.y + a3 * C.y + a4 * D.y) / dt);
  };
  double2 w[kMaxW];
#pragma unroll
  for (int q = 0; q < kMaxW; ++q) {
    w[q] = coef(q);
    if (q < n2) zt[size_t(q) * ncol + c] = w[q];
  }
  int base = 0;
  for (int i = 0; i < n2; ++i) {
    const int lo = P.ev_lo[i];
    while (base < lo) {
#pragma unroll
      for (int q = 0; q < kMaxW - 1; ++q) w[q] = w[q + 1];
      const int r = base + kMaxW;
      w[kMaxW - 1] = coef(r);
      if (r < n2) zt[size_t(r) * ncol + c] = w[kMaxW - 1];
      ++base;
    }
    const auto w0 = P.ev_w + size_t(i) * kMaxW;
    double2 acc = zero2();
#pragma unroll
    for (int q = 0; q < kMaxW; ++q) acc = fma2(w0[q], w[q], acc);
    V[size_t(i) * ncol + c] = acc;
  }
}

// ---------------------------------------------------------------------------
// Register-FFT plane kernels for the sizes of the workloads.  Line size N,
// T threads per line, radices R0..R3 (every radix divides N/T), PAD: one
// LDS pad slot every PAD positions (PAD < 0: the permutation of rf::padded).

// Several plans per size (V = 0, 1, 2: other thread counts, radix splits or stage orders) are compiled
// for the sizes below 768; the tile autotuner picks one by timing.  A size without alternatives uses its
// first plan for every V.
template <int N, int V>
struct LinePlanV : LinePlanV<N, 0> {};
#define LMVD_LINEPLAN(N_, V_, T_, R0_, R1_, R2_, R3_, PAD_)                                          \
  template <>                                                                                        \
  struct LinePlanV<N_, V_> {                                                                         \
    static constexpr int T = T_, R0 = R0_, R1 = R1_, R2 = R2_, R3 = R3_, PAD = PAD_;                 \
    static constexpr int E = N_ / T_;                                                                \
    static constexpr int RL = rf::Last<R0_, R1_, R2_, R3_>::value;                                   \
  };
LMVD_LINEPLAN(768, 0, 32, 24, 8, 4, 1, 24)
LMVD_LINEPLAN(384, 0, 32, 12, 4, 4, 2, 12)
LMVD_LINEPLAN(192, 0, 16, 12, 4, 4, 1, 12)
LMVD_LINEPLAN(192, 1, 8, 24, 8, 1, 1, 24)
LMVD_LINEPLAN(192, 2, 16, 12, 2, 2, 4, 12)
LMVD_LINEPLAN(144, 0, 12, 12, 12, 1, 1, 12)
LMVD_LINEPLAN(144, 1, 24, 6, 6, 2, 2, 6)
LMVD_LINEPLAN(144, 2, 6, 24, 6, 1, 1, 24)
LMVD_LINEPLAN(96, 0, 8, 12, 4, 2, 1, 12)
LMVD_LINEPLAN(96, 1, 4, 24, 4, 1, 1, 24)
LMVD_LINEPLAN(96, 2, 8, 12, 2, 4, 1, 12)
LMVD_LINEPLAN(72, 0, 6, 12, 6, 1, 1, 12)
LMVD_LINEPLAN(72, 1, 12, 6, 6, 2, 1, 6)
LMVD_LINEPLAN(72, 2, 3, 24, 3, 1, 1, 24)
LMVD_LINEPLAN(48, 0, 4, 12, 4, 1, 1, 12)
LMVD_LINEPLAN(48, 1, 8, 6, 2, 2, 2, 6)
LMVD_LINEPLAN(48, 2, 2, 24, 2, 1, 1, 24)
LMVD_LINEPLAN(36, 0, 3, 12, 3, 1, 1, 12)
LMVD_LINEPLAN(24, 0, 2, 12, 2, 1, 1, 12)
#undef LMVD_LINEPLAN
template <int N>
using LinePlan = LinePlanV<N, 0>;
// number of distinct z plans of a size
static constexpr int zplan_count(int n) {
  return (n == 192 || n == 144 || n == 96 || n == 72 || n == 48) ? 3 : 1;
}

// Tile code K of the register z kernels: K % 8 = D, the divisor of the lines per block, and K / 8 = V,
// the line plan.  LG = 256 / (T D) lines of T threads (lines = l, lane-fastest).  Fewer lines per block
// leave fewer idle lanes when the plan has few l-lines (small N1); the tile autotuner picks K per plan by
// timing.
template <int N, int K = 1>
struct ZShape {
  using LP = LinePlanV<N, K / 8>;
  static constexpr int T = LP::T;
  static constexpr int LG = kThreads / T / (K % 8);
  static_assert(LG >= 1, "z tile divisor too large for this transform");
  static constexpr int BASE = N + N / LP::PAD;
  // 8 lines: stride = 2 mod 32 keeps two neighbouring threads of each of the
  // 8 lines on distinct banks; otherwise an odd stride
  static constexpr int STRIDE = (LG == 8) ? (BASE + ((2 - BASE % 32) + 32) % 32) : (BASE | 1);
};
// x-line plans: full-length complex FFTs of m1 points, E = 12 per thread
template <int N>
struct XPlan;
#define LMVD_XPLAN(N_, T_, R0_, R1_, R2_, R3_, PAD_)                                                 \
  template <>                                                                                        \
  struct XPlan<N_> {                                                                                 \
    static constexpr int T = T_, R0 = R0_, R1 = R1_, R2 = R2_, R3 = R3_, PAD = PAD_;                 \
    static constexpr int E = N_ / T_;                                                                \
    static constexpr int RL = rf::Last<R0_, R1_, R2_, R3_>::value;                                   \
    static constexpr int BG = kThreads / T_;                     /* lines per block */               \
    static constexpr int STRIDE = PAD_ < 0 ? N_ : ((N_ + N_ / PAD_) + 1) / 2 * 2; /* doubles per line */ \
    static_assert(PAD_ > 0 || N_ % ((-PAD_) % 100 + 1) == 0, "the permutation must stay within the line");   \
  };
LMVD_XPLAN(768, 64, 12, 4, 4, 4, -231)  // LDS positions p ^ ((p >> 2) & 31)
LMVD_XPLAN(192, 16, 12, 4, 4, 1, 12)
LMVD_XPLAN(144, 12, 12, 12, 1, 1, 12)
LMVD_XPLAN(96, 8, 12, 4, 2, 1, 12)
LMVD_XPLAN(72, 6, 12, 6, 1, 1, 12)
LMVD_XPLAN(48, 4, 12, 4, 1, 1, 12)
#undef LMVD_XPLAN

// inverse z-FFT of size N = m3 of values at tau_j (optionally times i k1, the
// only multiplier that stays here: it is constant along a z line).
// grid (ceil(nl/LG), planes, nin), block LG*T (line index lane-fastest).
// EXACT: nn = 2N/3 - 1 (3/2 grid), so the zero-padded positions are known
// at compile time.
template <int N, bool EXACT, int D = 1>
__device__ __forceinline__ void zinv_r_body(const DevPlan& P, const unsigned bx, const unsigned by, const unsigned bz, const EvalArgs& A, double2* __restrict__ zbuf, int j0, int pb) {
  using LP = typename ZShape<N, D>::LP;
  using ZS = ZShape<N, D>;
  constexpr int T = LP::T, E = LP::E, LG = ZS::LG, RL = LP::RL;
  constexpr int NNX = 2 * N / 3 - 1, H3X = (NNX + 1) / 2, PADX = N - NNX;
  extern __shared__ double lds_d[];
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  const int f = bz, jj = by, j = j0 + jj, l = bx * LG + ll;
  const int nn = EXACT ? NNX : P.nn, nl = P.nl;
  const int h3 = EXACT ? H3X : (nn + 1) / 2, pad = EXACT ? PADX : N - nn;
  const EvalIn in = A.in[f];
  const bool lok = l < nl;
  const size_t ncol = size_t(nn) * nl;
  const double k1 = (lok && in.ma == MU_IK1) ? P.k1[l] : 0.0;
  const double2* src = in.a + size_t(j) * ncol + (lok ? l : 0);
  double2 v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int pos = tl + T * r;
    // compile-time zero when the whole r-slice lies in the padding
    const bool always_pad = EXACT && (T * r >= H3X) && (T * r + T - 1 < H3X + PADX);
    double2 val = zero2();
    if (!always_pad && lok && (pos < h3 || pos >= h3 + pad)) {
      const int ni = pos < h3 ? pos : pos - pad;
      val = src[size_t(ni) * nl];
      if (in.b) val = cadd(val, in.b[size_t(j) * ncol + size_t(ni) * nl + l]);
      if (in.ma == MU_IK3) val = apply_mult(MU_IK3, 0.0, P.k3[ni], val);
    }
    v[r] = val;
  }
  if (in.ma == MU_IK1) {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = make_double2(-k1 * v[r].y, k1 * v[r].x);
  }
  rf::run<N, T, 1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, ll * ZS::STRIDE, tl, P.fz.tw);
  if (lok) {
    double2* out = zbuf + (size_t(in.slot) * pb + jj) * size_t(N) * nl + l;
#pragma unroll
    for (int c = 0; c < E / RL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) out[size_t(tl + T * c + r * (N / RL)) * nl] = v[c * RL + r];
  }
}
template <int N, bool EXACT, int D>
__global__ void __launch_bounds__(kThreads) k_zinv_r(DevPlan P, EvalArgs A, double2* __restrict__ zbuf, int j0, int pb) {
  zinv_r_body<N, EXACT, D>(P, blockIdx.x, blockIdx.y, blockIdx.z, A, zbuf, j0, pb);
}

// forward z-FFT of size N = m3 and truncation to the retained n.
template <int N, int D = 1>
__device__ __forceinline__ void zfwd_r_body(const DevPlan& P, const unsigned bx, const unsigned by, const unsigned bz, const double2* __restrict__ obuf, const OutPtrs& V, int j0, int pb) {
  using LP = typename ZShape<N, D>::LP;
  using ZS = ZShape<N, D>;
  constexpr int T = LP::T, E = LP::E, LG = ZS::LG, RL = LP::RL;
  extern __shared__ double lds_d[];
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  const int g = bz, jj = by, l = bx * LG + ll;
  const int nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = N - nn;
  const bool lok = l < nl;
  const double2* in = obuf + (size_t(g) * pb + jj) * size_t(N) * nl + l;
  double2 v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = lok ? in[size_t(tl + T * r) * nl] : zero2();
  rf::run<N, T, -1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, ll * ZS::STRIDE, tl, P.fz.tw);
  if (lok) {
    double2* out = V.v[g] + size_t(j0 + jj) * nn * nl + l;
#pragma unroll
    for (int c = 0; c < E / RL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int pos = tl + T * c + r * (N / RL);
        if (pos < h3) out[size_t(pos) * nl] = v[c * RL + r];
        else if (pos >= h3 + pad) out[size_t(pos - pad) * nl] = v[c * RL + r];
      }
  }
}
template <int N, int D>
__global__ void __launch_bounds__(kThreads) k_zfwd_r(DevPlan P, const double2* __restrict__ obuf, OutPtrs V, int j0, int pb) {
  zfwd_r_body<N, D>(P, blockIdx.x, blockIdx.y, blockIdx.z, obuf, V, j0, pb);
}

// z kernels with one 64-thread group per line (12 points per thread) and 8
// lines per 512-thread block, the line index lane-fastest so that loads and
// stores of a wavefront cover 8 consecutive l (coalesced); exchanges move real
// and imaginary planes through LDS under block barriers, stage twiddles come
// from per-stage LDS tables.  Only the 768-point line has such a plan.
constexpr int kZWThreads = 512;
template <int N>
struct ZPlanW;
template <>
struct ZPlanW<768> {
  static constexpr int T = 64, R0 = 12, R1 = 4, R2 = 4, R3 = 4, PAD = 12, LG = 8;
  static constexpr int E = 768 / 64, RL = 4;
  static constexpr int STRIDE = 834;  // doubles per line: 768 + 768/12 padded to 2 mod 32
};

template <int N, bool EXACT>
__device__ __forceinline__ void zinv_w_body(const DevPlan& P, const unsigned bx, const unsigned by, const unsigned bz, const EvalArgs& A, double2* __restrict__ zbuf, int j0, int pb) {
  using ZP = ZPlanW<N>;
  constexpr int T = ZP::T, E = ZP::E, LG = ZP::LG, RL = ZP::RL;
  constexpr int NNX = 2 * N / 3 - 1, H3X = (NNX + 1) / 2, PADX = N - NNX;
  extern __shared__ double lds_d[];
  double2* twl = reinterpret_cast<double2*>(lds_d + LG * ZP::STRIDE);
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  // grid (fields, l groups, planes): the fields of one l group and plane are dispatched together, so
  // fields that read the same input (i k1 psi and i k3 psi) find it in the memory-side cache
  const int f = bx, jj = bz, j = j0 + jj, l = by * LG + ll;
  const int nn = EXACT ? NNX : P.nn, nl = P.nl;
  const int h3 = EXACT ? H3X : (nn + 1) / 2, pad = EXACT ? PADX : N - nn;
  rf::fill_stage_tw<N, ZP::R0, ZP::R1, ZP::R2, ZP::R3>(twl, P.fz.tw, tid, kZWThreads);
  const EvalIn in = A.in[f];
  const bool lok = l < nl;
  const size_t ncol = size_t(nn) * nl;
  const double k1 = (lok && in.ma == MU_IK1) ? P.k1[l] : 0.0;
  const size_t col0 = size_t(j) * ncol + (lok ? l : 0);
  double2 v[E];
  // all loads issued before any is used: absent points read mode 0 and are
  // then zeroed; the optional second field is a uniform branch around the batch
  auto load = [&](auto hasb) {
    const double2* __restrict__ sa = in.a + col0;
    const double2* __restrict__ sb = (hasb ? in.b : in.a) + col0;
    double2 xa[E], xb[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int pos = tl + T * r;
      const bool always_pad = EXACT && (T * r >= H3X) && (T * r + T - 1 < H3X + PADX);
      xa[r] = xb[r] = zero2();
      if (!always_pad) {
        const bool ok = lok && (pos < h3 || pos >= h3 + pad);
        const int ni = !ok ? 0 : (pos < h3 ? pos : pos - pad);
        xa[r] = sa[size_t(ni) * nl];
        if (hasb) xb[r] = sb[size_t(ni) * nl];
      }
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int pos = tl + T * r;
      const bool ok = lok && (pos < h3 || pos >= h3 + pad);
      v[r] = ok ? (hasb ? cadd(xa[r], xb[r]) : xa[r]) : zero2();
    }
    if (in.ma == MU_IK3) {  // i k3 of each point's z mode (zero-padded points stay zero)
#pragma unroll
      for (int r = 0; r < E; ++r) {
        const int pos = tl + T * r;
        const bool ok = lok && (pos < h3 || pos >= h3 + pad);
        if (ok) v[r] = apply_mult(MU_IK3, 0.0, P.k3[pos < h3 ? pos : pos - pad], v[r]);
      }
    }
  };
  if (in.b) load(std::true_type{});
  else load(std::false_type{});
  if (in.ma == MU_IK1) {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = make_double2(-k1 * v[r].y, k1 * v[r].x);
  }
  __syncthreads();  // twiddle tables
  rf::run_split<N, T, 1, ZP::R0, ZP::R1, ZP::R2, ZP::R3, ZP::PAD, true>(v, lds_d, ll * ZP::STRIDE, tl, twl);
  if (lok) {
    double2* out = zbuf + (size_t(in.slot) * pb + jj) * size_t(N) * nl + l;
#pragma unroll
    for (int c = 0; c < E / RL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) out[size_t(tl + T * c + r * (N / RL)) * nl] = v[c * RL + r];
  }
}
template <int N, bool EXACT>
__global__ void __launch_bounds__(kZWThreads) k_zinv_w(DevPlan P, EvalArgs A, double2* __restrict__ zbuf, int j0, int pb) {
  zinv_w_body<N, EXACT>(P, blockIdx.x, blockIdx.y, blockIdx.z, A, zbuf, j0, pb);
}

template <int N>
__device__ __forceinline__ void zfwd_w_body(const DevPlan& P, const unsigned bx, const unsigned by, const unsigned bz, const double2* __restrict__ obuf, const OutPtrs& V, int j0, int pb) {
  using ZP = ZPlanW<N>;
  constexpr int T = ZP::T, E = ZP::E, LG = ZP::LG, RL = ZP::RL;
  extern __shared__ double lds_d[];
  double2* twl = reinterpret_cast<double2*>(lds_d + LG * ZP::STRIDE);
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  // grid (fields, l groups, planes), as the inverse kernel
  const int g = bx, jj = bz, l = by * LG + ll;
  const int nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = N - nn;
  rf::fill_stage_tw<N, ZP::R0, ZP::R1, ZP::R2, ZP::R3>(twl, P.fz.tw, tid, kZWThreads);
  const bool lok = l < nl;
  const double2* in = obuf + (size_t(g) * pb + jj) * size_t(N) * nl + (lok ? l : 0);
  double2 v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = lok ? in[size_t(tl + T * r) * nl] : zero2();
  __syncthreads();  // twiddle tables
  rf::run_split<N, T, -1, ZP::R0, ZP::R1, ZP::R2, ZP::R3, ZP::PAD, true>(v, lds_d, ll * ZP::STRIDE, tl, twl);
  if (lok) {
    double2* out = V.v[g] + size_t(j0 + jj) * nn * nl + l;
#pragma unroll
    for (int c = 0; c < E / RL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int pos = tl + T * c + r * (N / RL);
        if (pos < h3) out[size_t(pos) * nl] = v[c * RL + r];
        else if (pos >= h3 + pad) out[size_t(pos - pad) * nl] = v[c * RL + r];
      }
  }
}
template <int N>
__global__ void __launch_bounds__(kZWThreads) k_zfwd_w(DevPlan P, const double2* __restrict__ obuf, OutPtrs V, int j0, int pb) {
  zfwd_w_body<N>(P, blockIdx.x, blockIdx.y, blockIdx.z, obuf, V, j0, pb);
}

// z filter of a non-final fixed-point iterate (eqs. y_k, disc_f).  A z line
// of x-spectral, z-physical values is transformed forward, the z modes
// outside the retained band are dropped, and it is transformed back: on
// interior planes these are the values at tau of the truncated, Neumann-
// projected iterate, because that projection interpolates the interior rows;
// k_wall then sets the two wall planes.  out = filter(in) + add (add already
// filtered, or null).  grid (ceil(nl/LG), planes); neither transform scales.
template <int N>
__device__ __forceinline__ void zfilt_w_body(const DevPlan& P, const unsigned bx, const unsigned by,
                                             const double2* __restrict__ in, const double2* __restrict__ add,
                                             double2* __restrict__ out) {
  using ZP = ZPlanW<N>;
  constexpr int T = ZP::T, E = ZP::E, LG = ZP::LG, RL = ZP::RL, EL = E / RL;
  extern __shared__ double lds_d[];
  double2* twl = reinterpret_cast<double2*>(lds_d + LG * ZP::STRIDE);
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  const int jj = by, l = bx * LG + ll;
  const int nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = N - nn;
  rf::fill_stage_tw<N, ZP::R0, ZP::R1, ZP::R2, ZP::R3>(twl, P.fz.tw, tid, kZWThreads);
  const bool lok = l < nl;
  const size_t base = size_t(jj) * N * nl + (lok ? l : 0);
  double2 v[E], w[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = lok ? in[base + size_t(tl + T * r) * nl] : zero2();
  __syncthreads();  // twiddle tables
  rf::run_split<N, T, -1, ZP::R0, ZP::R1, ZP::R2, ZP::R3, ZP::PAD, true>(v, lds_d, ll * ZP::STRIDE, tl, twl);
  // register c RL + r holds mode tl + T (c + EL r); natural order for the inverse, band only
#pragma unroll
  for (int c = 0; c < EL; ++c)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int pos = tl + T * (c + EL * r);
      w[c + EL * r] = (pos >= h3 && pos < h3 + pad) ? zero2() : v[c * RL + r];
    }
  rf::run_split<N, T, 1, ZP::R0, ZP::R1, ZP::R2, ZP::R3, ZP::PAD, true>(w, lds_d, ll * ZP::STRIDE, tl, twl);
  if (lok) {
#pragma unroll
    for (int c = 0; c < EL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const size_t e = base + size_t(tl + T * c + r * (N / RL)) * nl;
        const double2 x = w[c * RL + r];
        out[e] = add ? cadd(x, add[e]) : x;
      }
  }
}
template <int N>
__global__ void __launch_bounds__(kZWThreads) k_zfilt_w(DevPlan P, const double2* __restrict__ in,
                                                       const double2* __restrict__ add, double2* __restrict__ out) {
  zfilt_w_body<N>(P, blockIdx.x, blockIdx.y, in, add, out);
}
template <int N, int D = 1>
__device__ __forceinline__ void zfilt_r_body(const DevPlan& P, const unsigned bx, const unsigned by,
                                             const double2* __restrict__ in, const double2* __restrict__ add,
                                             double2* __restrict__ out) {
  using LP = typename ZShape<N, D>::LP;
  using ZS = ZShape<N, D>;
  constexpr int T = LP::T, E = LP::E, LG = ZS::LG, RL = LP::RL, EL = E / RL;
  extern __shared__ double lds_d[];
  const int tid = threadIdx.x;
  const int ll = tid % LG, tl = tid / LG;
  const int jj = by, l = bx * LG + ll;
  const int nn = P.nn, nl = P.nl, h3 = (nn + 1) / 2, pad = N - nn;
  const bool lok = l < nl;
  const size_t base = size_t(jj) * N * nl + (lok ? l : 0);
  double2 v[E], w[E];
#pragma unroll
  for (int r = 0; r < E; ++r) v[r] = lok ? in[base + size_t(tl + T * r) * nl] : zero2();
  rf::run<N, T, -1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, ll * ZS::STRIDE, tl, P.fz.tw);
#pragma unroll
  for (int c = 0; c < EL; ++c)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int pos = tl + T * (c + EL * r);
      w[c + EL * r] = (pos >= h3 && pos < h3 + pad) ? zero2() : v[c * RL + r];
    }
  __syncthreads();  // the forward transform's last LDS reads
  rf::run<N, T, 1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(w, lds_d, ll * ZS::STRIDE, tl, P.fz.tw);
  if (lok) {
#pragma unroll
    for (int c = 0; c < EL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const size_t e = base + size_t(tl + T * c + r * (N / RL)) * nl;
        const double2 x = w[c * RL + r];
        out[e] = add ? cadd(x, add[e]) : x;
      }
  }
}
template <int N, int D>
__global__ void __launch_bounds__(kThreads) k_zfilt_r(DevPlan P, const double2* __restrict__ in,
                                                     const double2* __restrict__ add, double2* __restrict__ out) {
  zfilt_r_body<N, D>(P, blockIdx.x, blockIdx.y, in, add, out);
}

// Wall planes of the filtered iterate: the Neumann projection's values at the
// wall rows are fixed sums of the interior values (weights wall_w, summed
// planes nearest each wall first).  zt: [n2][m3][nl] (all planes).
__device__ __forceinline__ void wall_body(const DevPlan& P, const unsigned bx, double2* zt) {
  const size_t ps = size_t(P.m3) * P.nl;
  const size_t e = size_t(bx) * blockDim.x + threadIdx.x;
  if (e >= ps) return;
  const int n2 = P.n2, k0 = P.wall_k0, k1 = P.wall_k1;
  const auto w0 = P.wall_w, w1 = P.wall_w + (k0 + 1);
  double2 a0 = zero2(), a1 = zero2();
  for (int d = 1; d <= k0; ++d) a0 = fma2(w0[d], zt[size_t(d) * ps + e], a0);
  for (int d = 1; d <= k1; ++d) a1 = fma2(w1[d], zt[size_t(n2 - 1 - d) * ps + e], a1);
  zt[e] = a0;
  zt[size_t(n2 - 1) * ps + e] = a1;
}
__global__ void __launch_bounds__(kThreads) k_wall(DevPlan P, double2* zt) { wall_body(P, blockIdx.x, zt); }

// Pointwise products of the x-pass.  Two real fields x, y travel through one
// complex FFT as x + i y, so a product of the pair needs no carried state.
// Input FFT I carries fields fa(I) and fb(I) (fb < 0: a single field, y = 0);
// in<I> folds the point values into the state s; output FFT Q carries
// fields ga(Q) and gb(Q) formed by out<Q>.
template <int PH>
struct Pair;

// inputs (zbuf slots) lap z, m1, z2, m2, z3, m3, z (z in slot 6, which the later phases of the substep
// leave alone, so the u, rho, C_ij pass reads it again):  R_z = (1/rho)(-m^d . grad z + rho D lap z)
template <>
struct Pair<PH_RZ> {
  static constexpr int NP = 4, NQ = 1, NST = 3;
  // pairs (d z / d x, lap z), (z, m1), (z2, m2), (z3, m3).  In a paired transform the rounding of each
  // field is of the order of the larger one.  lap z, by far the largest field, travels with a gradient
  // component, which reaches R_z only times the small m^d (and L z_t times m^c); a momentum paired with
  // lap z would carry that rounding into m . grad z, times the large gradient.  z's line is read twice:
  // for its x-derivative (formed mode by mode) and for z itself
  __device__ static constexpr int fa(int i) { return i < 2 ? 6 : 2 * i - 2; }
  __device__ static constexpr int fb(int i) { return i == 0 ? 0 : 2 * i - 1; }
  __device__ static constexpr bool dxa(int i) { return i == 0; }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan& P, double* s, double x, double y, double* a, size_t fs) {
    // a == nullptr on lines past the grid edge: nothing is written there
    if constexpr (I == 0) {  // x = d z / d x, y = lap z
      s[2] = x;
      s[1] = P.rhoD * y;
    } else if constexpr (I == 1) {  // x = z, y = m1
      const double rho = (P.rho_l * P.rho_h) / (P.rho_h - P.drho * x);
      s[0] = (P.rho_h - P.drho * x) * P.inv_rlrh;  // 1/rho
      s[1] -= s[2] * y;
      if (a) {
        a[3 * fs] = rho * rho * P.drho * P.inv_rlrh;
        a[0] = -s[0] * s[2];
      }
    } else {  // x = d z / d x_I, y = m_I
      s[1] -= x * y;
      if (a) a[(I - 1) * fs] = -s[0] * x;
    }
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) {
    return make_double2(s[1] * s[0], 0.0);
  }
};
// the same inputs with rho D = rho D(z): + (rho D)'(z) |grad z|^2 (div(rho D grad z) by the chain rule)
template <>
struct Pair<PH_RZV> {
  static constexpr int NP = 4, NQ = 1, NST = 3;
  // the pairs of PH_RZ
  __device__ static constexpr int fa(int i) { return Pair<PH_RZ>::fa(i); }
  __device__ static constexpr int fb(int i) { return Pair<PH_RZ>::fb(i); }
  __device__ static constexpr bool dxa(int i) { return Pair<PH_RZ>::dxa(i); }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan& P, double* s, double x, double y, double* a, size_t fs) {
    if constexpr (I == 0) {  // x = d z / d x, y = lap z (kept until rho D(z) is known)
      s[2] = x;
      s[1] = y;
    } else if constexpr (I == 1) {  // x = z, y = m1
      const double rho = (P.rho_l * P.rho_h) / (P.rho_h - P.drho * x);
      double k, dk;
      rhod_of(P, x, rho, k, dk);
      s[0] = (P.rho_h - P.drho * x) * P.inv_rlrh;  // 1/rho
      s[1] = fma(dk * s[2], s[2], k * s[1] - s[2] * y);
      if (a) {
        a[3 * fs] = rho * rho * P.drho * P.inv_rlrh;
        a[0] = -s[0] * s[2];
      }
      s[2] = dk;
    } else {  // x = d z / d x_I, y = m_I
      s[1] = fma(s[2] * x, x, s[1] - x * y);
      if (a) a[(I - 1) * fs] = -s[0] * x;
    }
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) {
    return make_double2(s[1] * s[0], 0.0);
  }
};
// inputs (zbuf slots) S_a, S_b, S_c in slots 0..2 and z in slot 6 -> tau = mu(z) S (fields 0..2); run
// once per group of three strain components, so that four doubles of state per point stay in registers
template <>
struct Pair<PH_TAU> {
  static constexpr int NP = 2, NQ = 2, NST = 4;
  // pairs (z, S_a), (S_b, S_c)
  __device__ static constexpr int fa(int i) { return i == 0 ? 6 : 1; }
  __device__ static constexpr int fb(int i) { return i == 0 ? 0 : 2; }
  __device__ static constexpr bool dxa(int) { return false; }
  __device__ static constexpr int ga(int q) { return q == 0 ? 0 : 2; }
  __device__ static constexpr int gb(int q) { return q == 0 ? 1 : -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan& P, double* s, double x, double y, double*, size_t) {
    if constexpr (I == 0) {
      s[0] = mu_of(P, x);
      s[1] = s[0] * y;
    } else {
      s[2] = s[0] * x;
      s[3] = s[0] * y;
    }
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) {
    if constexpr (Q == 0) return make_double2(s[1], s[2]);
    else return make_double2(s[3], 0.0);
  }
};
template <>
struct Pair<PH_L> {  // inputs m1c, m2c, m3c:  L z_t = -(1/rho) grad z . m^c = g . m^c
  static constexpr int NP = 2, NQ = 1, NST = 1;
  __device__ static constexpr int fa(int i) { return 2 * i; }
  __device__ static constexpr int fb(int i) { return i == 0 ? 1 : -1; }
  __device__ static constexpr bool dxa(int) { return false; }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan&, double* s, double x, double y, double* a, size_t fs) {
    if constexpr (I == 0) s[0] = a[0] * x + a[fs] * y;
    else s[0] += a[2 * fs] * x;
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) { return make_double2(s[0], 0.0); }
};
template <>
struct Pair<PH_RHOT> {  // input z_t:  rho_t = f'(z) z_t
  static constexpr int NP = 1, NQ = 1, NST = 1;
  __device__ static constexpr int fa(int) { return 0; }
  __device__ static constexpr int fb(int) { return -1; }
  __device__ static constexpr bool dxa(int) { return false; }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan&, double* s, double x, double, double* a, size_t fs) {
    s[0] = a[3 * fs] * x;
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) { return make_double2(s[0], 0.0); }
};
// inputs (zbuf slots) m1, m2, m3, and z in slot 6 -> u1, u2, u3, rho, C11, C12, C13, C22, C23, C33 (fields 0..9)
template <>
struct Pair<PH_VEL> {
  static constexpr int NP = 2, NQ = 5, NST = 4;
  // pairs (z, m1), (m2, m3)
  __device__ static constexpr int fa(int i) { return i == 0 ? 6 : 1; }
  __device__ static constexpr int fb(int i) { return i == 0 ? 0 : 2; }
  __device__ static constexpr bool dxa(int) { return false; }
  // output pairs ordered so that m1, then m2, then m3 is last used early
  // (the transforms are unrolled): (C11, C12), (C13, u1), (C22, C23), (u2, rho), (C33, u3)
  __device__ static constexpr int ga(int q) { return q == 0 ? 4 : q == 1 ? 6 : q == 2 ? 7 : q == 3 ? 1 : 9; }
  __device__ static constexpr int gb(int q) { return q == 0 ? 5 : q == 1 ? 0 : q == 2 ? 8 : q == 3 ? 3 : 2; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan& P, double* s, double x, double y, double*, size_t) {
    if constexpr (I == 0) {
      s[0] = P.rho_h - P.drho * x;  // rl rh / rho
      s[1] = y;
    } else {
      s[2] = x;
      s[3] = y;
    }
  }
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan& P, const double* s) {
    const double ir = s[0] * P.inv_rlrh;
    if constexpr (Q == 0) return make_double2(-s[1] * (s[1] * ir), -s[1] * (s[2] * ir));
    else if constexpr (Q == 1) return make_double2(-s[1] * (s[3] * ir), s[1] * ir);
    else if constexpr (Q == 2) return make_double2(-s[2] * (s[2] * ir), -s[2] * (s[3] * ir));
    else if constexpr (Q == 3) return make_double2(s[2] * ir, (P.rho_l * P.rho_h) / s[0]);
    else return make_double2(-s[3] * (s[3] * ir), s[3] * ir);
  }
};
template <>
struct Pair<PH_TOPHYS> {  // one input, written out on the physical grid
  static constexpr int NP = 1, NQ = 0, NST = 1;
  __device__ static constexpr int fa(int) { return 0; }
  __device__ static constexpr int fb(int) { return -1; }
  __device__ static constexpr bool dxa(int) { return false; }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan&, double*, double, double, double*, size_t) {}
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double*) { return zero2(); }
};
template <>
struct Pair<PH_FROMPHYS> {  // one output, read from the physical grid
  static constexpr int NP = 0, NQ = 1, NST = 1;
  __device__ static constexpr int fa(int) { return 0; }
  __device__ static constexpr int fb(int) { return -1; }
  __device__ static constexpr bool dxa(int) { return false; }
  __device__ static constexpr int ga(int q) { return q; }
  __device__ static constexpr int gb(int) { return -1; }
  template <int I>
  __device__ __forceinline__ static void in(const DevPlan&, double*, double, double, double*, size_t) {}
  template <int Q>
  __device__ __forceinline__ static double2 out(const DevPlan&, const double* s) { return make_double2(s[0], 0.0); }
};

// state update of input FFT I (runtime index i) on every point of the thread;
// point q of the line (position tl + T q) sits in register slot
// v[c*RL + r] with q = c + r*EL after an inverse transform
template <class S, int I, int E, int RL, int NST, int T>
__device__ __forceinline__ void pair_in(const DevPlan& P, int i, double (&st)[NST][E], const double2* v, double* ap,
                                        size_t fs) {
  if constexpr (I < S::NP) {
    if (i == I) {
      constexpr int EL = E / RL;
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int q = c + r * EL;
          double s[NST];
#pragma unroll
          for (int k = 0; k < NST; ++k) s[k] = st[k][q];
          S::template in<I>(P, s, v[c * RL + r].x, v[c * RL + r].y, ap + T * q, fs);
#pragma unroll
          for (int k = 0; k < NST; ++k) st[k][q] = s[k];
        }
    } else {
      pair_in<S, I + 1, E, RL, NST, T>(P, i, st, v, ap, fs);
    }
  }
}
template <class S, int Q, int E, int NST>
__device__ __forceinline__ void pair_out(const DevPlan& P, int q, const double (&st)[NST][E], double2* v) {
  if constexpr (Q < S::NQ) {
    if (q == Q) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        double s[NST];
#pragma unroll
        for (int k = 0; k < NST; ++k) s[k] = st[k][e];
        v[e] = S::template out<Q>(P, s);
      }
    } else {
      pair_out<S, Q + 1, E, NST>(P, q, st, v);
    }
  }
}

// Restores the range 0 <= t < T of a lane index made opaque to the compiler,
// so that positions t + (multiple of the padding period) fold to immediate
// LDS offsets.
template <int T>
__device__ __forceinline__ int lane_in_line(int t) {
  if constexpr ((T & (T - 1)) == 0) {
    return t & (T - 1);
  } else {
    __builtin_assume(t >= 0 && t < T);
    return t;
  }
}

// Transform input Z = X + i Y of a line pair from the N/3 retained modes of
// X (at XA) and Y (at XB; absent when !HASB): Z_k = X_k + i Y_k for k < N/3
// (imaginary parts of X_0, Y_0 dropped), Z_{N-k} = conj(X_k) + i conj(Y_k),
// zero in between.  oka / okb false: that line is absent (its pointer must
// still be readable).  N/3 and 2N/3 are multiples of T, so the class of each
// point is known at compile time; every load is issued before any is used.
// DXA: X is replaced by its x-derivative, X_k -> i k1[k] X_k (k1: the x wavenumbers).
template <int N, int T, bool HASB, bool DXA = false>
__device__ __forceinline__ void herm_pair_load(double2* v, const double2* __restrict__ XA,
                                               const double2* __restrict__ XB, int tl, bool oka, bool okb,
                                               const double* __restrict__ k1 = nullptr) {
  constexpr int E = N / T, NL = N / 3;
  static_assert(NL % T == 0, "retained band must be whole rows of T points");
  double2 a[E], b[E];
  double ka[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    a[r] = b[r] = zero2();
    ka[r] = 0.0;
    if (T * r + T <= NL) {
      a[r] = XA[tl + T * r];
      if (HASB) b[r] = XB[tl + T * r];
      if (DXA) ka[r] = k1[tl + T * r];
    } else if (T * r >= N - NL) {
      const int m = N - T * r - tl;  // in [1, N/3]
      const int mm = m < NL ? m : 0;
      a[r] = XA[mm];
      if (HASB) b[r] = XB[mm];
      if (DXA) ka[r] = k1[mm];
    }
  }
  if (DXA) {
#pragma unroll
    for (int r = 0; r < E; ++r) a[r] = make_double2(-ka[r] * a[r].y, ka[r] * a[r].x);
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    double2 xa = oka ? a[r] : zero2();
    double2 xb = (HASB && okb) ? b[r] : zero2();
    double2 z = zero2();
    if (T * r + T <= NL) {
      if (r == 0 && tl == 0) {
        xa.y = 0.0;
        xb.y = 0.0;
      }
      z = make_double2(xa.x - xb.y, xa.y + xb.x);
    } else if (T * r >= N - NL) {
      if (N - T * r - tl < NL) z = make_double2(xa.x + xb.y, xb.x - xa.y);
    }
    v[r] = z;
  }
}

// x-pass: per (plane, z line b) inverse x-FFTs of the inputs, products,
// forward x-FFTs of the outputs, m1 = N points, retained modes l < N/3.
// Spectral line X_l (l < N/3) of a real field; a pair X, Y enters one
// transform as Z_l = X_l + i Y_l, Z_{N-l} = conj(X_l) + i conj(Y_l), with
// the real parts of X_0, Y_0 (what the Hermitian extension keeps).  An
// output pair u + i v with transform W splits as U_k = (W_k + conj W_{N-k})/2,
// V_k = (W_k - conj W_{N-k})/(2i).  grid (ceil(m3/BG), planes), block BG*T.
template <int PH, int N>
__device__ __forceinline__ void xpair_body(const DevPlan& P, const unsigned bx, const unsigned by,
                                           const double2* __restrict__ zbuf,
                                           double2* __restrict__ obuf, int pb, double* phys_out,
                                           const double* phys_in, int j0, double* __restrict__ aux) {
  using LP = XPlan<N>;
  using S = Pair<PH>;
  constexpr int T = LP::T, E = LP::E, RL = LP::RL, EL = E / RL, BG = LP::BG, NL = N / 3;
  static_assert(E == 12 && NL % T == 0, "x plans hold 12 points per thread, N/3 retained modes");
  constexpr int QL = NL / T;  // points q < QL hold retained modes k = tl + T q < N/3
  extern __shared__ double lds_d[];
  double2* twl = reinterpret_cast<double2*>(lds_d + BG * LP::STRIDE);
  const int tid = threadIdx.x;
  // one line per wavefront when T is the wave size: the line index is then
  // uniform, and so are the line's base addresses (scalar registers)
  const int tl = tid % T, line = (T == 64) ? __builtin_amdgcn_readfirstlane(tid / T) : tid / T;
  const int jj = by, b = bx * BG + line;
  const int M3 = P.m3;
  const bool bok = b < M3;
  const int bb = bok ? b : 0;
  rf::fill_stage_tw<N, LP::R0, LP::R1, LP::R2, LP::R3>(twl, P.xtw, tid, BG * T);
  __syncthreads();
  const int base = line * LP::STRIDE;
  double st[S::NST][E];
#pragma unroll
  for (int k = 0; k < S::NST; ++k)
#pragma unroll
    for (int q = 0; q < E; ++q) st[k][q] = 0.0;
  double2 v[E];
#pragma unroll 1
  for (int i = 0; i < S::NP; ++i) {
    // opaque per iteration: keeps the compiler from hoisting every LDS address
    // and twiddle of the transform out of the loop (register pressure)
    int tlx = tl, basex = base;
    asm volatile("" : "+v"(tlx), "+v"(basex));
    tlx = lane_in_line<T>(tlx);
    const int fa = S::fa(i), fb = S::fb(i);
    const double2* XA = zbuf + ((size_t(fa) * pb + jj) * M3 + bb) * NL;
    const double2* XB = zbuf + ((size_t(fb < 0 ? fa : fb) * pb + jj) * M3 + bb) * NL;
    if (fb >= 0 && S::dxa(i)) herm_pair_load<N, T, true, true>(v, XA, XB, tlx, bok, bok, P.k1);
    else if (fb >= 0) herm_pair_load<N, T, true>(v, XA, XB, tlx, bok, bok);
    else herm_pair_load<N, T, false>(v, XA, XA, tlx, bok, bok);
    rf::run_split<N, T, 1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, basex, tlx, twl);
    if constexpr (PH == PH_TOPHYS) {
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int q = c + r * EL;
          if (bok) phys_out[(size_t(j0 + jj) * M3 + b) * P.m1 + tl + T * q] = v[c * RL + r].x;
        }
    } else {
      // aux point q of this thread: ap[T q], fields fs apart
      double* ap = (aux && (bok || (PH != PH_RZ && PH != PH_RZV))) ? aux + (size_t(j0 + jj) * M3 + bb) * P.m1 + tl : nullptr;
      pair_in<S, 0, E, RL, S::NST, T>(P, i, st, v, ap, size_t(P.n2) * M3 * P.m1);
    }
  }
  if constexpr (PH == PH_FROMPHYS) {
    const double* src = phys_in + (size_t(j0 + jj) * M3 + bb) * P.m1 + tl;
#pragma unroll
    for (int q = 0; q < E; ++q) st[0][q] = bok ? src[T * q] : 0.0;
  }
  const double scale = 1.0 / (double(P.m1) * double(M3));
  // unrolled: with several outputs the state of a point dies output by output
#pragma unroll
  for (int q = 0; q < S::NQ; ++q) {
    int tlx = tl, basex = base;
    asm volatile("" : "+v"(tlx), "+v"(basex));
    tlx = lane_in_line<T>(tlx);
    pair_out<S, 0, E, S::NST>(P, q, st, v);
    rf::run_split<N, T, -1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, basex, tlx, twl);
    // W at point q' = c + r EL (k = tl + T q')
    const int ga = S::ga(q), gb = S::gb(q);
    double2* YA = obuf + ((size_t(ga) * pb + jj) * M3 + bb) * NL;
    if (gb < 0) {
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r)
          if (c + r * EL < QL && bok) YA[tlx + T * (c + r * EL)] = cscale(v[c * RL + r], scale);
    } else {
      double2* YB = obuf + ((size_t(gb) * pb + jj) * M3 + bb) * NL;
      // partners W_{N-k} of the retained k sit at point 0 and the points above N - N/3
      double pre[QL], pim[QL];
      rf::line_sync<T>();
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int qq = c + r * EL;
          if (qq == 0 || T * qq + T - 1 > N - NL) lds_d[basex + rf::padded<LP::PAD>(tlx + T * qq)] = v[c * RL + r].x;
        }
      rf::line_sync<T>();
#pragma unroll
      for (int qq = 0; qq < QL; ++qq) pre[qq] = lds_d[basex + rf::padded<LP::PAD>((N - tlx - T * qq) % N)];
      rf::line_sync<T>();
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int qq = c + r * EL;
          if (qq == 0 || T * qq + T - 1 > N - NL) lds_d[basex + rf::padded<LP::PAD>(tlx + T * qq)] = v[c * RL + r].y;
        }
      rf::line_sync<T>();
#pragma unroll
      for (int qq = 0; qq < QL; ++qq) pim[qq] = lds_d[basex + rf::padded<LP::PAD>((N - tlx - T * qq) % N)];
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int qq = c + r * EL;
          if (qq < QL && bok) {
            const double2 w = v[c * RL + r];
            const double hs = 0.5 * scale;
            YA[tlx + T * qq] = make_double2(hs * (w.x + pre[qq]), hs * (w.y - pim[qq]));
            YB[tlx + T * qq] = make_double2(hs * (w.y + pim[qq]), -hs * (w.x - pre[qq]));
          }
        }
    }
  }
}

// x-pass with line pairing, for phases whose inputs are products of one field
// with physical aux fields (L z_t and rho_t): every transform carries one
// field on two neighbouring z lines b0, b1 as x(b0) + i x(b1), so a single
// field costs half a transform.  Traits: input I is field I; in<I> folds the
// point value x into the point state s (aux a, field stride fs); output Q is
// field Q, formed by out<Q>.
template <int PH>
struct LineOp;
template <>
struct LineOp<PH_L> {  // inputs m1c, m2c, m3c:  L z_t = g . m^c (aux fields g1, g2, g3)
  static constexpr int NP = 3, NQ = 1;
  __device__ static constexpr int aux_field(int i) { return i; }
  template <int I>
  __device__ __forceinline__ static void in(double& s, double x, double a) {
    if constexpr (I == 0) s = a * x;
    else s += a * x;
  }
};
template <>
struct LineOp<PH_RHOT> {  // input z_t:  rho_t = f'(z) z_t (aux field f')
  static constexpr int NP = 1, NQ = 1;
  __device__ static constexpr int aux_field(int) { return 3; }
  template <int I>
  __device__ __forceinline__ static void in(double& s, double x, double a) {
    s = a * x;
  }
};

// a0, a1: the aux field of input i at point 0 of lines b0, b1 (point q at T q)
template <class S, int I, int E, int RL, int T>
__device__ __forceinline__ void line_in(int i, double (&s0)[E], double (&s1)[E], const double2* v,
                                        const double* __restrict__ a0, const double* __restrict__ a1) {
  if constexpr (I < S::NP) {
    if (i == I) {
      constexpr int EL = E / RL;
#pragma unroll
      for (int c = 0; c < EL; ++c)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
          const int q = c + r * EL;
          S::template in<I>(s0[q], v[c * RL + r].x, a0[T * q]);
          S::template in<I>(s1[q], v[c * RL + r].y, a1[T * q]);
        }
    } else {
      line_in<S, I + 1, E, RL, T>(i, s0, s1, v, a0, a1);
    }
  }
}

template <int PH, int N>
__device__ __forceinline__ void xline_body(const DevPlan& P, const unsigned bx, const unsigned by, const double2* __restrict__ zbuf, double2* __restrict__ obuf, int pb, int j0, const double* __restrict__ aux) {
  using LP = XPlan<N>;
  using S = LineOp<PH>;
  constexpr int T = LP::T, E = LP::E, RL = LP::RL, EL = E / RL, BG = LP::BG, NL = N / 3;
  static_assert(E == 12 && NL % T == 0, "x plans hold 12 points per thread, N/3 retained modes");
  constexpr int QL = NL / T;
  extern __shared__ double lds_d[];
  double2* twl = reinterpret_cast<double2*>(lds_d + BG * LP::STRIDE);
  const int tid = threadIdx.x;
  const int tl = tid % T, grp = (T == 64) ? __builtin_amdgcn_readfirstlane(tid / T) : tid / T;
  const int jj = by;
  const int b0 = 2 * (bx * BG + grp), b1 = b0 + 1;
  const int M3 = P.m3;
  const bool ok0 = b0 < M3, ok1 = b1 < M3;
  const int c0 = ok0 ? b0 : 0, c1 = ok1 ? b1 : 0;
  rf::fill_stage_tw<N, LP::R0, LP::R1, LP::R2, LP::R3>(twl, P.xtw, tid, BG * T);
  __syncthreads();
  const int base = grp * LP::STRIDE;
  const size_t fs = size_t(P.n2) * M3 * P.m1;
  const double* a0 = aux + (size_t(j0 + jj) * M3 + c0) * P.m1 + tl;
  const double* a1 = aux + (size_t(j0 + jj) * M3 + c1) * P.m1 + tl;
  double s0[E], s1[E];
#pragma unroll
  for (int q = 0; q < E; ++q) s0[q] = s1[q] = 0.0;
  double2 v[E];
#pragma unroll 1
  for (int i = 0; i < S::NP; ++i) {
    int tlx = tl, basex = base;
    asm volatile("" : "+v"(tlx), "+v"(basex));
    tlx = lane_in_line<T>(tlx);
    const double2* XA = zbuf + ((size_t(i) * pb + jj) * M3 + c0) * NL;
    const double2* XB = zbuf + ((size_t(i) * pb + jj) * M3 + c1) * NL;
    herm_pair_load<N, T, true>(v, XA, XB, tlx, ok0, ok1);
    rf::run_split<N, T, 1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, basex, tlx, twl);
    const double* ai0 = a0 + S::aux_field(i) * fs;
    const double* ai1 = a1 + S::aux_field(i) * fs;
    asm volatile("" : "+v"(ai0), "+v"(ai1));
    line_in<S, 0, E, RL, T>(i, s0, s1, v, ai0, ai1);
  }
  const double scale = 1.0 / (double(P.m1) * double(M3));
#pragma unroll 1
  for (int q = 0; q < S::NQ; ++q) {
    int tlx = tl, basex = base;
    asm volatile("" : "+v"(tlx), "+v"(basex));
    tlx = lane_in_line<T>(tlx);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = make_double2(s0[e], s1[e]);
    rf::run_split<N, T, -1, LP::R0, LP::R1, LP::R2, LP::R3, LP::PAD>(v, lds_d, basex, tlx, twl);
    double2* YA = obuf + ((size_t(q) * pb + jj) * M3 + c0) * NL;
    double2* YB = obuf + ((size_t(q) * pb + jj) * M3 + c1) * NL;
    // partners W_{N-k} of the retained k sit at point 0 and the points above N - N/3
    double pre[QL], pim[QL];
    rf::line_sync<T>();
#pragma unroll
    for (int c = 0; c < EL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int qq = c + r * EL;
        if (qq == 0 || T * qq + T - 1 > N - NL) lds_d[basex + rf::padded<LP::PAD>(tlx + T * qq)] = v[c * RL + r].x;
      }
    rf::line_sync<T>();
#pragma unroll
    for (int qq = 0; qq < QL; ++qq) pre[qq] = lds_d[basex + rf::padded<LP::PAD>((N - tlx - T * qq) % N)];
    rf::line_sync<T>();
#pragma unroll
    for (int c = 0; c < EL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int qq = c + r * EL;
        if (qq == 0 || T * qq + T - 1 > N - NL) lds_d[basex + rf::padded<LP::PAD>(tlx + T * qq)] = v[c * RL + r].y;
      }
    rf::line_sync<T>();
#pragma unroll
    for (int qq = 0; qq < QL; ++qq) pim[qq] = lds_d[basex + rf::padded<LP::PAD>((N - tlx - T * qq) % N)];
#pragma unroll
    for (int c = 0; c < EL; ++c)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int qq = c + r * EL;
        if (qq < QL) {
          const double2 w = v[c * RL + r];
          const double hs = 0.5 * scale;
          if (ok0) YA[tlx + T * qq] = make_double2(hs * (w.x + pre[qq]), hs * (w.y - pim[qq]));
          if (ok1) YB[tlx + T * qq] = make_double2(hs * (w.y + pim[qq]), -hs * (w.x - pre[qq]));
        }
      }
  }
}
template <int PH, int N>
__global__ void __launch_bounds__(kThreads) k_xline(DevPlan P, const double2* __restrict__ zbuf, double2* __restrict__ obuf, int pb, int j0, const double* __restrict__ aux) {
  xline_body<PH, N>(P, blockIdx.x, blockIdx.y, zbuf, obuf, pb, j0, aux);
}

// Kernels of the x-pass.  The u, rho, C_ij pass keeps four values per point
// across five output transforms; its register budget is capped at two waves
// per SIMD (the rest spills), which measured faster than one wave per SIMD.
template <int PH, int N>
__global__ void __launch_bounds__(kThreads) k_xpair(DevPlan P, const double2* __restrict__ zbuf,
                                                   double2* __restrict__ obuf, int pb, double* phys_out,
                                                   const double* phys_in, int j0, double* __restrict__ aux) {
  xpair_body<PH, N>(P, blockIdx.x, blockIdx.y, zbuf, obuf, pb, phys_out, phys_in, j0, aux);
}
template <int PH, int N>
__global__ void __launch_bounds__(kThreads, 2) k_xpair_w2(DevPlan P, const double2* __restrict__ zbuf,
                                                         double2* __restrict__ obuf, int pb, double* phys_out,
                                                         const double* phys_in, int j0, double* __restrict__ aux) {
  xpair_body<PH, N>(P, blockIdx.x, blockIdx.y, zbuf, obuf, pb, phys_out, phys_in, j0, aux);
}


// ---------------------------------------------------------------------------
// column kernel: projection values -> B coefficients with a shared no-pivot LU
// (kind 0 interpolation, 1 Dirichlet rows, 2 Neumann rows).  One thread per
// column; forward sweep stores L^{-1} b in `out`, backward sweep overwrites it.

// Rows read this many steps ahead of the sweeps' dependent chains (see the m^c kernel's rings).
constexpr int kProjPre = 4;

template <int EPI>
__device__ __forceinline__ void proj_body(const DevPlan& P, int c, int kind, const double2* in, double2* out,
                                          const double2* __restrict__ add, const double2* __restrict__ z,
                                          const double2* __restrict__ zt_prev, double2* __restrict__ z_out,
                                          double2* __restrict__ vals_out, double2* __restrict__ vals_out1,
                                          int stage, int ncol) {
  if (c >= ncol) return;
  constexpr int D = kProjPre;
  const int n2 = P.n2;
  const int nfull = n2 - n2 % D;
  const auto L = P.lu_l + size_t(kind) * n2 * kMaxBand;
  const auto U = P.lu_u + size_t(kind) * n2 * (kMaxBand + 1);
  const auto Ui = P.lu_uinv + size_t(kind) * n2;
  double2 ring[kMaxBand];
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) ring[m] = zero2();
  // band rows of the next step, read while the current step runs (scalar loads, one row ahead)
  double cnx[kMaxBand + 1];
  auto load_l = [&](int i) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) cnx[m] = L[min(i, n2 - 1) * kMaxBand + m];
  };
  // ascending L sweep; slot d of pv holds the next input row i = d (mod D)
  auto fwd = [&](int i, double2 b) __attribute__((always_inline)) {
    double lc[kMaxBand];
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) lc[m] = cnx[m];
    load_l(i + 1);
    if (kind != 0 && (i == 0 || i == n2 - 1)) b = zero2();
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) b = fma2(-lc[m], ring[m], b);
    out[size_t(i) * ncol + c] = b;
#pragma unroll
    for (int m = kMaxBand - 1; m > 0; --m) ring[m] = ring[m - 1];
    ring[0] = b;
  };
  {
    load_l(0);
    double2 pv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) pv[d] = in[size_t(min(d, n2 - 1)) * ncol + c];
    for (int i0 = 0; i0 < nfull; i0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = i0 + d;
        fwd(i, pv[d]);
        pv[d] = in[size_t(min(i + D, n2 - 1)) * ncol + c];
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (nfull + d < n2) fwd(nfull + d, pv[d]);
  }
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) ring[m] = zero2();
  // window of the final output rows i .. i+kMaxW-1 for the E0 values (vals_out)
  double2 win[kMaxW];
#pragma unroll
  for (int q = 0; q < kMaxW; ++q) win[q] = zero2();
  // descending U sweep; the rows it reads (the L-sweep result, and for the fixed-point epilogues the
  // added field, z and the previous stage's z_t) come through rings of D slots like the ascending one
  const double2* ztp = (stage != 0) ? zt_prev : z;  // read unconditionally, used at stage 1 only
  struct Rows {
    double2 y, a, z0, zp;
  };
  auto load = [&](Rows& r, int i) __attribute__((always_inline)) {
    const size_t e = size_t(i) * ncol + c;
    r.y = out[e];
    if (EPI != EPI_STORE) r.a = add[e];
    if (EPI == EPI_ADD_ZUPDATE) {
      r.z0 = z[e];
      r.zp = ztp[e];
    }
  };
  auto load_u = [&](int i) __attribute__((always_inline)) {
    i = max(i, 0);
#pragma unroll
    for (int q = 0; q < kMaxBand; ++q) cnx[q] = U[i * (kMaxBand + 1) + q + 1];
    cnx[kMaxBand] = Ui[i];
  };
  auto bwd = [&](int i, const Rows& r) __attribute__((always_inline)) {
    double uc[kMaxBand + 1];
#pragma unroll
    for (int q = 0; q <= kMaxBand; ++q) uc[q] = cnx[q];
    load_u(i - 1);
    double2 y = r.y;
#pragma unroll
    for (int q = 0; q < kMaxBand; ++q) y = fma2(-uc[q], ring[q], y);
    const double2 x = cscale(y, uc[kMaxBand]);
#pragma unroll
    for (int q = kMaxBand - 1; q > 0; --q) ring[q] = ring[q - 1];
    ring[0] = x;
    const size_t e = size_t(i) * ncol + c;
    const double2 fin = (EPI == EPI_STORE) ? x : cadd(x, r.a);
    // a non-final fixed-point iterate (EPI_ADD) is consumed only through its emitted values
    if (EPI != EPI_ADD) out[e] = fin;
    if (vals_out) {
#pragma unroll
      for (int q = kMaxW - 1; q > 0; --q) win[q] = win[q - 1];
      win[0] = fin;
      const int first = P.emit_first[i], cnt = P.emit_cnt[i];
      for (int t = 0; t < cnt; ++t) {
        const auto w0 = P.ev_w + size_t(first + t) * kMaxW;
        double2 acc = zero2();
#pragma unroll
        for (int q = 0; q < kMaxW; ++q) acc = fma2(w0[q], win[q], acc);
        vals_out[size_t(first + t) * ncol + c] = acc;
        if (vals_out1) {
          const auto w1 = P.ev_w + (size_t(n2) + first + t) * kMaxW;
          double2 acc1 = zero2();
#pragma unroll
          for (int q = 0; q < kMaxW; ++q) acc1 = fma2(w1[q], win[q], acc1);
          vals_out1[size_t(first + t) * ncol + c] = acc1;
        }
      }
    }
    if (EPI == EPI_ADD_ZUPDATE) {
      const double2 zt = fin;
      double2 zn;
      if (stage == 0) {
        zn = fma2(0.5 * P.dt, zt, r.z0);
      } else {
        const double2 dz = make_double2(zt.x - 0.5 * r.zp.x, zt.y - 0.5 * r.zp.y);
        zn = fma2(P.dt, dz, r.z0);
      }
      z_out[e] = zn;
    }
  };
  {
    load_u(n2 - 1);
    Rows pr[D];  // slot d: step t = d (mod D) of the sweep, row i = n2 - 1 - t
#pragma unroll
    for (int d = 0; d < D; ++d) load(pr[d], max(n2 - 1 - d, 0));
    for (int t0 = 0; t0 < nfull; t0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = n2 - 1 - (t0 + d);
        bwd(i, pr[d]);
        load(pr[d], max(i - D, 0));
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (nfull + d < n2) bwd(n2 - 1 - (nfull + d), pr[d]);
  }
}

template <int EPI>
__global__ void __launch_bounds__(kThreads) k_proj(DevPlan P, int kind, const double2* in, double2* out,
                                                   const double2* __restrict__ add, const double2* __restrict__ z,
                                                   const double2* __restrict__ zt_prev, double2* __restrict__ z_out,
                                                   double2* __restrict__ vals_out, double2* __restrict__ vals_out1,
                                                   int stage, int ncol) {
  proj_body<EPI>(P, int(blockIdx.x * blockDim.x + threadIdx.x), kind, in, out, add, z, zt_prev, z_out, vals_out,
                 vals_out1, stage, ncol);
}

// Independent plain projections of the same kind in one launch (field blockIdx.y).
struct ProjBatch {
  const double2* in[3];
  double2* out[3];
};
__global__ void __launch_bounds__(kThreads) k_proj3(DevPlan P, int kind, ProjBatch B, int ncol) {
  const int f = blockIdx.y;
  proj_body<EPI_STORE>(P, int(blockIdx.x * blockDim.x + threadIdx.x), kind, B.in[f], B.out[f], nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, 0, ncol);
}

// ---------------------------------------------------------------------------
// column kernel: T_ij = C_ij + tau_ij at the Greville points, their
// interpolation, and their share of the right-hand sides of Omega2 and phi2
// (eqs. om, phi with the body force).  tau_ij = mu (d_j u_i + d_i u_j)
// - 2/3 mu theta delta_ij is linear in u, so its values follow from the
// projected velocity u_hat directly (i k1, d/dy, i k3): the same numbers the
// 3/2-grid round trip of the derivative fields would give, since the forward
// transform inverts the inverse one on the retained modes.
// With N_i = i k1 T_i1 + d/dy T_i2 + i k3 T_i3 (T symmetric):
//   RHS_Omega2 = i k3 N1 - i k1 N3
//   RHS_phi2   = -k^2 N2 - d/dy (i k1 N1 + i k3 N3) + k^2 g rho
// GROUP 0 (T11, T12, T13) writes its part of both at tau; GROUP 1 (T22, T23,
// T33) adds its part and the buoyancy term.  The ascending sweep reads u_hat
// through register windows (every coefficient once) and forms the L solve of
// the interpolation; the descending U solve keeps a window of T_hat rows and
// emits every tau row whose band starts at the current row.  Only the
// (0, 0) column keeps T12 / T23 coefficients (for the plane means).
// W: register window (>= B-spline order), LB: band of the interpolation LU.
template <int W>
struct RowWin {
  double2 w[W];
  int base;
  __device__ __forceinline__ void init(const double2* __restrict__ src, size_t ncol, size_t c, int rows) {
    base = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) w[q] = (q < rows) ? src[size_t(q) * ncol + c] : zero2();
  }
  __device__ __forceinline__ void advance(const double2* __restrict__ src, size_t ncol, size_t c, int rows, int lo) {
    while (base < lo) {
#pragma unroll
      for (int q = 0; q < W - 1; ++q) w[q] = w[q + 1];
      const int r = base + W;
      w[W - 1] = (r < rows) ? src[size_t(r) * ncol + c] : zero2();
      ++base;
    }
  }
  __device__ __forceinline__ double2 dot(cptr<double> wt) const {
    double2 acc = zero2();
#pragma unroll
    for (int q = 0; q < W; ++q) acc = fma2(wt[q], w[q], acc);
    return acc;
  }
};

// VARMU: mu = mu(z); tau_ij was formed on the physical grid (mu(z) S_ij) and its values at tau are read
// from Ta, Tb, Tc (which the sweep then overwrites, row by row, with its own intermediates); u is not read.
template <int GROUP, int W, int LB, bool VARMU = false>
__device__ __forceinline__ void flux_body(const DevPlan& P, const unsigned bx, const double2* __restrict__ Ca,
                                          const double2* __restrict__ Cb, const double2* __restrict__ Cc,
                                          const double2* __restrict__ u1, const double2* __restrict__ u2,
                                          const double2* __restrict__ u3, double2* Ta, double2* Tb, double2* Tc,
                                          double2* RO, double2* RP, const double2* __restrict__ rhov) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2;
  const size_t ncol = size_t(nn) * nl;
  const size_t c = size_t(bx) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double k1 = P.k1[c % nl], k3 = P.k3[c / nl], ksq = k1 * k1 + k3 * k3;
  const double mu = P.mu, th = (2.0 / 3.0) * P.mu;
  const auto L = P.lu_l;
  const auto U = P.lu_u;
  const auto Ui = P.lu_uinv;
  {
    RowWin<W> w1, w2, w3;
    if constexpr (!VARMU) {
      w1.init(u1, ncol, c, n2);
      w2.init(u2, ncol, c, n2);
      w3.init(u3, ncol, c, n2);
    }
    double2 ra[LB], rb[LB], rc[LB];
#pragma unroll
    for (int m = 0; m < LB; ++m) ra[m] = rb[m] = rc[m] = zero2();
    for (int i = 0; i < n2; ++i) {
      const size_t e = size_t(i) * ncol + c;
      double2 ba, bb, bc;
      if constexpr (VARMU) {
        ba = cadd(Ca[e], Ta[e]);
        bb = cadd(Cb[e], Tb[e]);
        bc = cadd(Cc[e], Tc[e]);
      } else {
        const int lo = P.ev_lo[i];
        w1.advance(u1, ncol, c, n2, lo);
        w2.advance(u2, ncol, c, n2, lo);
        w3.advance(u3, ncol, c, n2, lo);
        const auto e0 = P.ev_w + size_t(i) * kMaxW;
        const auto e1 = P.ev_w + (size_t(n2) + i) * kMaxW;
        double2 s0[3] = {w1.dot(e0), w2.dot(e0), w3.dot(e0)};
        double2 s1[3] = {w1.dot(e1), w2.dot(e1), w3.dot(e1)};
        // d[a][b] = d u_a / d x_b at tau_i
        double2 d[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          d[a][0] = times_i(cscale(s0[a], k1));
          d[a][1] = s1[a];
          d[a][2] = times_i(cscale(s0[a], k3));
        }
        const double2 theta = cadd(cadd(d[0][0], d[1][1]), d[2][2]);
        if (GROUP == 0) {
          ba = cadd(Ca[e], make_double2(2 * mu * d[0][0].x - th * theta.x, 2 * mu * d[0][0].y - th * theta.y));
          bb = cadd(Cb[e], cscale(cadd(d[0][1], d[1][0]), mu));
          bc = cadd(Cc[e], cscale(cadd(d[0][2], d[2][0]), mu));
        } else {
          ba = cadd(Ca[e], make_double2(2 * mu * d[1][1].x - th * theta.x, 2 * mu * d[1][1].y - th * theta.y));
          bb = cadd(Cb[e], cscale(cadd(d[1][2], d[2][1]), mu));
          bc = cadd(Cc[e], make_double2(2 * mu * d[2][2].x - th * theta.x, 2 * mu * d[2][2].y - th * theta.y));
        }
      }
#pragma unroll
      for (int m = 0; m < LB; ++m) {
        const double lm = L[i * kMaxBand + m];
        ba = fma2(-lm, ra[m], ba);
        bb = fma2(-lm, rb[m], bb);
        bc = fma2(-lm, rc[m], bc);
      }
      Ta[e] = ba;
      Tb[e] = bb;
      Tc[e] = bc;
#pragma unroll
      for (int m = LB - 1; m > 0; --m) {
        ra[m] = ra[m - 1];
        rb[m] = rb[m - 1];
        rc[m] = rc[m - 1];
      }
      ra[0] = ba;
      rb[0] = bb;
      rc[0] = bc;
    }
  }
  double2 wa[W], wb[W], wc[W];  // T_hat rows i .. i+W-1
#pragma unroll
  for (int q = 0; q < W; ++q) wa[q] = wb[q] = wc[q] = zero2();
  const double k1k3 = k1 * k3;
  for (int i = n2 - 1; i >= 0; --i) {
    const size_t e = size_t(i) * ncol + c;
    double2 ya = Ta[e], yb = Tb[e], yc = Tc[e];
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const double u = U[i * (kMaxBand + 1) + q + 1];
      ya = fma2(-u, wa[q], ya);
      yb = fma2(-u, wb[q], yb);
      yc = fma2(-u, wc[q], yc);
    }
#pragma unroll
    for (int q = W - 1; q > 0; --q) {
      wa[q] = wa[q - 1];
      wb[q] = wb[q - 1];
      wc[q] = wc[q - 1];
    }
    wa[0] = cscale(ya, Ui[i]);
    wb[0] = cscale(yb, Ui[i]);
    wc[0] = cscale(yc, Ui[i]);
    if (c == 0) Tb[e] = wb[0];
    const int first = P.emit_first[i], cnt = P.emit_cnt[i];
    for (int t = 0; t < cnt; ++t) {
      const int r = first + t;
      const auto e0 = P.ev_w + size_t(r) * kMaxW;
      const auto e1 = P.ev_w + (size_t(n2) + r) * kMaxW;
      const auto e2 = P.ev_w + (size_t(2 * n2) + r) * kMaxW;
      double2 a0 = zero2(), a1 = zero2(), b0 = zero2(), b1 = zero2(), b2 = zero2(), c0 = zero2(), c1 = zero2();
#pragma unroll
      for (int q = 0; q < W; ++q) {
        a0 = fma2(e0[q], wa[q], a0);
        a1 = fma2(e1[q], wa[q], a1);
        b0 = fma2(e0[q], wb[q], b0);
        b1 = fma2(e1[q], wb[q], b1);
        b2 = fma2(e2[q], wb[q], b2);
        c0 = fma2(e0[q], wc[q], c0);
        c1 = fma2(e1[q], wc[q], c1);
      }
      const size_t o = size_t(r) * ncol + c;
      double2 om, ph;
      if (GROUP == 0) {  // a = T11, b = T12, c = T13
        // -k1 k3 E0 T11 + i k3 E1 T12 + (k1^2 - k3^2) E0 T13
        om = cadd(cadd(cscale(a0, -k1k3), times_i(cscale(b1, k3))), cscale(c0, k1 * k1 - k3 * k3));
        // k1^2 E1 T11 - i k1 (k^2 E0 T12 + E2 T12) + 2 k1 k3 E1 T13
        const double2 t12 = make_double2(ksq * b0.x + b2.x, ksq * b0.y + b2.y);
        ph = cadd(csub(cscale(a1, k1 * k1), times_i(cscale(t12, k1))), cscale(c1, 2.0 * k1k3));
      } else {  // a = T22, b = T23, c = T33
        // -i k1 E1 T23 + k1 k3 E0 T33
        om = cadd(RO[o], csub(cscale(c0, k1k3), times_i(cscale(b1, k1))));
        // -k^2 E1 T22 - i k3 (k^2 E0 T23 + E2 T23) + k3^2 E1 T33 + k^2 g rho
        const double2 t23 = make_double2(ksq * b0.x + b2.x, ksq * b0.y + b2.y);
        const double2 rv = rhov[o];
        ph = cadd(RP[o], cadd(csub(cscale(c1, k3 * k3), times_i(cscale(t23, k3))),
                              make_double2(ksq * (P.g * rv.x - a1.x), ksq * (P.g * rv.y - a1.y))));
      }
      RO[o] = om;
      RP[o] = ph;
    }
  }
}
template <int GROUP, int W, int LB, bool VARMU>
__global__ void __launch_bounds__(kThreads) k_flux(DevPlan P, const double2* __restrict__ Ca,
                                  const double2* __restrict__ Cb, const double2* __restrict__ Cc,
                                  const double2* __restrict__ u1, const double2* __restrict__ u2,
                                  const double2* __restrict__ u3, double2* Ta, double2* Tb, double2* Tc, double2* RO,
                                  double2* RP, const double2* __restrict__ rhov) {
  flux_body<GROUP, W, LB, VARMU>(P, blockIdx.x, Ca, Cb, Cc, u1, u2, u3, Ta, Tb, Tc, RO, RP, rhov);
}

// column kernel (variable viscosity): the rate-of-strain values S_ij = d_j u_i + d_i u_j - 2/3 theta
// delta_ij (i <= j) at the Greville points from the projected velocity u_hat (i k1, d/dy, i k3), for the
// physical-grid product tau_ij = mu(z) S_ij
struct SixPtr {
  double2* v[6];
};
template <int W>
__device__ __forceinline__ void strain_body(const DevPlan& P, const unsigned bx, const double2* __restrict__ u1,
                                            const double2* __restrict__ u2, const double2* __restrict__ u3,
                                            const SixPtr& S) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2;
  const size_t ncol = size_t(nn) * nl;
  const size_t c = size_t(bx) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double k1 = P.k1[c % nl], k3 = P.k3[c / nl];
  RowWin<W> w1, w2, w3;
  w1.init(u1, ncol, c, n2);
  w2.init(u2, ncol, c, n2);
  w3.init(u3, ncol, c, n2);
  for (int i = 0; i < n2; ++i) {
    const int lo = P.ev_lo[i];
    w1.advance(u1, ncol, c, n2, lo);
    w2.advance(u2, ncol, c, n2, lo);
    w3.advance(u3, ncol, c, n2, lo);
    const auto e0 = P.ev_w + size_t(i) * kMaxW;
    const auto e1 = P.ev_w + (size_t(n2) + i) * kMaxW;
    const double2 s0[3] = {w1.dot(e0), w2.dot(e0), w3.dot(e0)};
    const double2 s1[3] = {w1.dot(e1), w2.dot(e1), w3.dot(e1)};
    double2 d[3][3];  // d u_a / d x_b at tau_i
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d[a][0] = times_i(cscale(s0[a], k1));
      d[a][1] = s1[a];
      d[a][2] = times_i(cscale(s0[a], k3));
    }
    const double2 th = cscale(cadd(cadd(d[0][0], d[1][1]), d[2][2]), 2.0 / 3.0);
    const size_t e = size_t(i) * ncol + c;
    S.v[0][e] = csub(cscale(d[0][0], 2.0), th);
    S.v[1][e] = cadd(d[0][1], d[1][0]);
    S.v[2][e] = cadd(d[0][2], d[2][0]);
    S.v[3][e] = csub(cscale(d[1][1], 2.0), th);
    S.v[4][e] = cadd(d[1][2], d[2][1]);
    S.v[5][e] = csub(cscale(d[2][2], 2.0), th);
  }
}
template <int W>
__global__ void __launch_bounds__(kThreads) k_strain(DevPlan P, const double2* __restrict__ u1,
                                                     const double2* __restrict__ u2,
                                                     const double2* __restrict__ u3, SixPtr S) {
  strain_body<W>(P, blockIdx.x, u1, u2, u3, S);
}

// ---------------------------------------------------------------------------
// column kernel: the per-wavenumber systems A(k) c = r,
//   A(k) = E*_2 - k^2 E*_0 at the interior tau*, Robin rows
//   k m2 - m2' = 0 (bottom), k m2 + m2' = 0 (top) (eqs. phi_poisson, bc_both),
// LU without pivoting formed on the fly in the forward sweep; the U rows go to
// a scratch array, read back by the backward sweep.  One thread solves the
// pair (l, n), (l, -n), which share k.  The backward sweep emits the
// reconstructions:
//   MODE 0 (m^d):  r = G0 phi2;      m1 = (i k1 D*c - i k3 Omega2)/k^2,
//                                    m3 = (i k3 D*c + i k1 Omega2)/k^2  (eq. md_recon)
//   MODE 1 (m^c):  r = -G1 rho_t;    m_par = (i/k)(rho_t + D*c)        (eqs. COM_fourier, CF_fourier)
// The (0,0) thread handles the plane mean: m^d = (<m>1, 0, <m>3); for m^c
// D*c = -<rho_t>, c_top = 0 (eq. mc_mean with <m2>(+L2/2) = 0).

template <int MODE, int LO, int UP>
__global__ void __launch_bounds__(kThreads) k_solveA(DevPlan P, const double2* __restrict__ in1,
                                                     const double2* __restrict__ in2, const double* __restrict__ m1bar,
                                                     const double* __restrict__ m3bar, double2* __restrict__ c2,
                                                     double2* __restrict__ o1, double2* __restrict__ o3,
                                                     double* __restrict__ uscr) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const int half = (nn + 1) / 2;
  const int npairs = nl * half;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npairs) return;
  const int l = t % nl, pp = t / nl;
  const size_t ncol = size_t(nn) * nl;
  const size_t cA = size_t(pp) * nl + l;
  const bool two = pp > 0;
  const size_t cB = two ? size_t(nn - pp) * nl + l : cA;
  const double k1 = P.k1[l], k3 = P.k3[pp];
  const double ksq = k1 * k1 + k3 * k3;
  if (ksq == 0.0) {
    // plane mean
    if (MODE == 0) {
      for (int i = 0; i < N; ++i) c2[size_t(i) * ncol] = zero2();
      for (int i = 0; i < n2; ++i) {
        o1[size_t(i) * ncol] = make_double2(m1bar[i], 0.0);
        o3[size_t(i) * ncol] = make_double2(m3bar[i], 0.0);
      }
    } else {
      double2 c = zero2();
      c2[size_t(n2) * ncol] = c;
      for (int i = n2 - 1; i >= 0; --i) {
        const double2 r = in1[size_t(i) * ncol];
        c = make_double2(c.x + r.x / P.dstar[i], c.y + r.y / P.dstar[i]);
        c2[size_t(i) * ncol] = c;
        o1[size_t(i) * ncol] = zero2();
      }
    }
    return;
  }
  const double k = sqrt(ksq);
  constexpr int W = LO + UP + 1;
  double uw[LO][UP];       // U rows i-1..i-LO, entries for columns r+1..r+UP
  double uinvw[LO];
  double2 ya[LO], yb[LO];
#pragma unroll
  for (int m = 0; m < LO; ++m) {
    uinvw[m] = 0.0;
    ya[m] = yb[m] = zero2();
#pragma unroll
    for (int q = 0; q < UP; ++q) uw[m][q] = 0.0;
  }
  const auto elo = P.es_lo;
  const auto ew = P.es_w;
  const int Ns = n2 + 1;
  const auto Gw = P.gs_w + (MODE == 0 ? 0 : size_t(Ns) * kMaxW);
  const auto Glo = P.gs_lo + (MODE == 0 ? 0 : Ns);
  const double gsign = (MODE == 0) ? 1.0 : -1.0;
  const size_t ustride = size_t(npairs);
  for (int i = 0; i < N; ++i) {
    double a[W];
    const int lo0 = elo[i], lo1 = elo[Ns + i], lo2 = elo[2 * Ns + i];
    const bool robin = (i == 0 || i == n2);
    const double sg = (i == 0) ? -1.0 : 1.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int col = i - LO + w;
      const int q0 = col - lo0, q1 = col - lo1, q2 = col - lo2;
      const double e0 = (q0 >= 0 && q0 < kMaxW) ? ew[(size_t(i)) * kMaxW + q0] : 0.0;
      if (robin) {
        const double e1 = (q1 >= 0 && q1 < kMaxW) ? ew[(size_t(Ns) + i) * kMaxW + q1] : 0.0;
        a[w] = k * e0 + sg * e1;
      } else {
        const double e2 = (q2 >= 0 && q2 < kMaxW) ? ew[(size_t(2 * Ns) + i) * kMaxW + q2] : 0.0;
        a[w] = e2 - ksq * e0;
      }
    }
    double2 ra = zero2(), rb = zero2();
    if (!robin) {
      const int glo = Glo[i];
      const auto gw = Gw + size_t(i) * kMaxW;
#pragma unroll
      for (int q = 0; q < kMaxW; ++q) {
        const int r = glo + q;
        if (gw[q] != 0.0 && r < n2) {
          ra = fma2(gsign * gw[q], in1[size_t(r) * ncol + cA], ra);
          if (two) rb = fma2(gsign * gw[q], in1[size_t(r) * ncol + cB], rb);
        }
      }
    }
    // eliminate columns i-LO .. i-1 with the stored pivot rows
#pragma unroll
    for (int m = LO; m >= 1; --m) {
      const double lm = a[LO - m] * uinvw[m - 1];
#pragma unroll
      for (int q = 1; q <= UP; ++q) {
        if (LO - m + q < W) a[LO - m + q] -= lm * uw[m - 1][q - 1];
      }
      ra = fma2(-lm, ya[m - 1], ra);
      rb = fma2(-lm, yb[m - 1], rb);
    }
    const double uinv = 1.0 / a[LO];
    double* us = uscr + size_t(i) * (UP + 1) * ustride + t;
    us[0] = uinv;
#pragma unroll
    for (int q = 1; q <= UP; ++q) us[q * ustride] = a[LO + q];
    c2[size_t(i) * ncol + cA] = ra;
    if (two) c2[size_t(i) * ncol + cB] = rb;
#pragma unroll
    for (int m = LO - 1; m > 0; --m) {
      uinvw[m] = uinvw[m - 1];
      ya[m] = ya[m - 1];
      yb[m] = yb[m - 1];
#pragma unroll
      for (int q = 0; q < UP; ++q) uw[m][q] = uw[m - 1][q];
    }
    uinvw[0] = uinv;
    ya[0] = ra;
    yb[0] = rb;
#pragma unroll
    for (int q = 0; q < UP; ++q) uw[0][q] = a[LO + 1 + q];
  }
  // backward sweep
  double2 xa[UP], xb[UP];
#pragma unroll
  for (int q = 0; q < UP; ++q) xa[q] = xb[q] = zero2();
  const double ik = 1.0 / k, iksq = 1.0 / ksq;
  for (int i = N - 1; i >= 0; --i) {
    const double* us = uscr + size_t(i) * (UP + 1) * ustride + t;
    double2 ya_ = c2[size_t(i) * ncol + cA];
    double2 yb_ = two ? c2[size_t(i) * ncol + cB] : zero2();
#pragma unroll
    for (int q = 1; q <= UP; ++q) {
      const double u = us[q * ustride];
      ya_ = fma2(-u, xa[q - 1], ya_);
      yb_ = fma2(-u, xb[q - 1], yb_);
    }
    const double uinv = us[0];
    const double2 xA = cscale(ya_, uinv), xB = cscale(yb_, uinv);
    c2[size_t(i) * ncol + cA] = xA;
    if (two) c2[size_t(i) * ncol + cB] = xB;
    if (i < n2) {
      const double ds = P.dstar[i];
      // (D* c)_i = dstar_i (c_{i+1} - c_i); c_{i+1} = xa[0] before the shift
      const double2 DA = make_double2(ds * (xa[0].x - xA.x), ds * (xa[0].y - xA.y));
      const double2 DB = make_double2(ds * (xb[0].x - xB.x), ds * (xb[0].y - xB.y));
      const size_t eA = size_t(i) * ncol + cA, eB = size_t(i) * ncol + cB;
      if (MODE == 0) {
        const double2 OA = in2[eA];
        // (i k1 D - i k3 Omega)/k^2, (i k3 D + i k1 Omega)/k^2
        o1[eA] = cscale(times_i(make_double2(k1 * DA.x - k3 * OA.x, k1 * DA.y - k3 * OA.y)), iksq);
        o3[eA] = cscale(times_i(make_double2(k3 * DA.x + k1 * OA.x, k3 * DA.y + k1 * OA.y)), iksq);
        if (two) {
          const double2 OB = in2[eB];
          const double k3b = -k3;
          o1[eB] = cscale(times_i(make_double2(k1 * DB.x - k3b * OB.x, k1 * DB.y - k3b * OB.y)), iksq);
          o3[eB] = cscale(times_i(make_double2(k3b * DB.x + k1 * OB.x, k3b * DB.y + k1 * OB.y)), iksq);
        }
      } else {
        const double2 RA = in1[eA];
        o1[eA] = cscale(times_i(cadd(RA, DA)), ik);
        if (two) o1[eB] = cscale(times_i(cadd(in1[eB], DB)), ik);
      }
    }
#pragma unroll
    for (int q = UP - 1; q > 0; --q) {
      xa[q] = xa[q - 1];
      xb[q] = xb[q - 1];
    }
    xa[0] = xA;
    xb[0] = xB;
  }
}

// ---------------------------------------------------------------------------
// A(k) factors, computed once per plan: bottom-up elimination without
// pivoting (rows n2 .. 0), one thread per pair (l, +-n) (A depends on k only).
// Row i keeps nm_i <= UA multipliers (of rows i+1 .. i+nm_i), its ns_i <= LA
// entries left of the diagonal and 1/pivot (nm_i, ns_i: the structure of A,
// from the plan), at fac[(fac_off[i] + slot) * npairs + t].  A(k) = E*_2 - k^2 E*_0 at interior tau*, Robin rows
// k m2 - m2' (bottom), k m2 + m2' (top) (eqs. phi_poisson, bc_both).
// Every row is checked as it is eliminated: with s the largest magnitude of the row of A, the pivot must
// reach kPivotMin s and no entry of the eliminated row may exceed growth_max s (a row that fails, or
// holds a NaN, counts in stats[0]); stats[1] and stats[2] receive the largest growth and the smallest
// pivot ratio of all pairs (bit patterns of positive floats, which order like the values).
constexpr double kPivotMin = 1e-12;
constexpr double kGrowthMax = 1e4;  // default growth limit of the check at plan creation
template <int LA, int UA>
__global__ void __launch_bounds__(kThreads) k_factor_ul(DevPlan P, double* __restrict__ fac, double growth_max,
                                                        unsigned* __restrict__ stats) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const int npairs = nl * ((nn + 1) / 2);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npairs) return;
  const int l = t % nl, pp = t / nl;
  const double k1 = P.k1[l], k3 = P.k3[pp];
  const double ksq = k1 * k1 + k3 * k3;
  constexpr int W = LA + UA + 1;
  if (ksq == 0.0) {
    for (int i = 0; i < N; ++i) {
      const int ns = P.fac_nm[i] + P.fac_ns[i] + 1;
      for (int q = 0; q < ns; ++q) fac[(size_t(P.fac_off[i]) + q) * npairs + t] = 0.0;
    }
    return;
  }
  const double k = sqrt(ksq);
  const int Ns = n2 + 1;
  const auto elo = P.es_lo;
  const auto ew = P.es_w;
  double piv[UA][LA];  // entries left of the diagonal of pivot rows i+1 .. i+UA
  double pinv[UA];
  unsigned bad = 0;
  double gmax = 0.0, rmin = 1.0 / 0.0;
#pragma unroll
  for (int m = 0; m < UA; ++m) {
    pinv[m] = 0.0;
#pragma unroll
    for (int q = 0; q < LA; ++q) piv[m][q] = 0.0;
  }
  for (int i = N - 1; i >= 0; --i) {
    double a[W];  // a[w] = A[i][i - LA + w]
    const int lo0 = elo[i], lo1 = elo[Ns + i], lo2 = elo[2 * Ns + i];
    const bool robin = (i == 0 || i == n2);
    const double sg = (i == 0) ? -1.0 : 1.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int col = i - LA + w;
      const int q0 = col - lo0, q1 = col - lo1, q2 = col - lo2;
      const double e0 = (q0 >= 0 && q0 < kMaxW) ? ew[size_t(i) * kMaxW + q0] : 0.0;
      if (robin) {
        const double e1 = (q1 >= 0 && q1 < kMaxW) ? ew[(size_t(Ns) + i) * kMaxW + q1] : 0.0;
        a[w] = k * e0 + sg * e1;
      } else {
        const double e2 = (q2 >= 0 && q2 < kMaxW) ? ew[(size_t(2 * Ns) + i) * kMaxW + q2] : 0.0;
        a[w] = e2 - ksq * e0;
      }
    }
    const int nm = P.fac_nm[i], ns = P.fac_ns[i];
    double* f = fac + size_t(P.fac_off[i]) * npairs + t;
    double rs = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) rs = fmax(rs, fabs(a[w]));
    // eliminate columns i+UA .. i+1 with pivot rows i+UA .. i+1 (farthest first)
#pragma unroll
    for (int m = UA; m >= 1; --m) {
      const double lm = a[LA + m] * pinv[m - 1];
#pragma unroll
      for (int q = 1; q <= LA; ++q) a[LA + m - q] -= lm * piv[m - 1][q - 1];
      if (m <= nm) f[size_t(m - 1) * npairs] = lm;
    }
    double big = 0.0;
#pragma unroll
    for (int w = 0; w <= LA; ++w) big = fmax(big, fabs(a[w]));
    const double growth = big / rs, ratio = fabs(a[LA]) / rs;
    if (!(ratio >= kPivotMin) || !(growth <= growth_max)) ++bad;
    gmax = fmax(gmax, growth);
    rmin = fmin(rmin, ratio);
    const double dinv = 1.0 / a[LA];
#pragma unroll
    for (int q = 1; q <= LA; ++q)
      if (q <= ns) f[size_t(nm + q - 1) * npairs] = a[LA - q];
    f[size_t(nm + ns) * npairs] = dinv;
#pragma unroll
    for (int m = UA - 1; m > 0; --m) {
      pinv[m] = pinv[m - 1];
#pragma unroll
      for (int q = 0; q < LA; ++q) piv[m][q] = piv[m - 1][q];
    }
    pinv[0] = dinv;
#pragma unroll
    for (int q = 1; q <= LA; ++q) piv[0][q - 1] = a[LA - q];
  }
  if (bad) atomicAdd(&stats[0], bad);
  atomicMax(&stats[1], __float_as_uint(float(fmin(gmax, 3.0e38))));
  atomicMin(&stats[2], __float_as_uint(float(rmin)));
}

// ---------------------------------------------------------------------------
// column kernel: m^c of one fixed-point iterate from the rho_t values at tau
// (eqs. COM_fourier, CF_fourier, mc_mean), one thread per column; the two
// columns (l, n), (l, -n) of a pair are neighbouring lanes and share the
// factors of A(k).
//   1. interpolation rho_t = P0 (values): ascending L sweep (scratch yp),
//   2. descending U sweep; every interior tau* row i whose G1 band starts at
//      the current row gets r_i = -G1 rho_t at once and enters the bottom-up
//      forward sweep of A(k) c = r (scratch yt); Robin rows have r = 0,
//   3. ascending back substitution for c (the B* coefficients of m2); every
//      tau row whose F0/F1 band is complete emits the values
//        m2 = F0 c,  m_par = (i/k)(rho_t + F1 c),  m1 = (k1/k) m_par,  m3 = (k3/k) m_par
//      or, without V3 (an iterate whose m^c is used only by L z_t), m2 and the potential
//      psi = (rho_t + F1 c) / k^2 in V1, of which m1 = i k1 psi and m3 = i k3 psi (the inverse z
//      transform applies the factors), so one value field less is written and read
//      (F1 = E0 D*, so F1 c = E0 D* c and E0 rho_t is the input value itself).
// Plane mean (k = 0): D* c = -<rho_t>, c_top = 0, m1 = m3 = 0.
// With d1 (final iterate) the m^d values are added and the coefficients
// c2 = c, mparc = (i/k)(rho_t + D* c) and rhoc = rho_t are written.
// LDS layout of the tables a sweep of k_mc reads (doubles, then ints), per
// phase; phase 2: U rows of the interpolation (LB), 1/pivots, G1 rows,
// G1 emission counts, factor row counts and offsets; phase 3:
// F0/F1 emission weights, emission starts and counts, factor row structure.
struct McLds {
  int n2, N, lb;
  __host__ __device__ int p2_doubles() const { return n2 * lb + n2 + N * kMaxW + n2; }
  __host__ __device__ int p2_ints() const { return n2 + 2 * N; }
  __host__ __device__ int p3_doubles() const { return 2 * n2 * kMaxW + n2; }
  __host__ __device__ int p3_ints() const { return 2 * N + 3 * N; }
  __host__ __device__ size_t bytes() const {
    const size_t a = size_t(p2_doubles()) * 8 + size_t(p2_ints()) * 4;
    const size_t b = size_t(p3_doubles()) * 8 + size_t(p3_ints()) * 4;
    return a > b ? a : b;
  }
};

// STAGE: the row tables of phases 2 and 3 are copied to LDS at the start of
// each phase (every row of every column reads them with the same index, so
// LDS latency replaces a scalar-cache miss per row); threads without a
// column still take part in the copies and barriers.
template <int LA, int UA, int LB, bool STAGE>
__device__ __forceinline__ void mc_body(const DevPlan& P, const unsigned bx, const double2* __restrict__ vals,
                                        double2* yp, double2* yt, const double2* __restrict__ d1,
                                        const double2* __restrict__ d2, const double2* __restrict__ d3,
                                        double2* __restrict__ V1, double2* __restrict__ V2, double2* __restrict__ V3,
                                        double2* rhoc, double2* __restrict__ c2, double2* __restrict__ mparc) {
  extern __shared__ double lds_d[];
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const int half = (nn + 1) / 2, npairs = nl * half;
  const int t = bx * blockDim.x + threadIdx.x;
  const int pr = t >> 1, side = t & 1;
  const int l = pr % nl, pp = pr / nl;
  const bool active = pr < npairs && !(side == 1 && pp == 0);
  if (!STAGE && !active) return;
  const int ni = active ? (side ? nn - pp : pp) : 0;
  const size_t ncol = size_t(nn) * nl, c = size_t(ni) * nl + (active ? l : 0);
  const double k1 = active ? P.k1[l] : 1.0, k3 = P.k3[ni], ksq = k1 * k1 + k3 * k3;
  const bool mean = (ksq == 0.0);
  const double ik = mean ? 0.0 : 1.0 / sqrt(ksq);
  const double* fac = P.fac + (active ? pr : 0);
  const McLds lay{n2, N, LB};
  // 1. ascending sweep of the interpolation projection (rows loaded kPreMc ahead)
  if (active) {
    double2 ring[LB];
#pragma unroll
    for (int m = 0; m < LB; ++m) ring[m] = zero2();
    double lnx[LB];  // band row of the next step, read one row ahead (scalar loads)
    auto load_l = [&](int i) __attribute__((always_inline)) {
#pragma unroll
      for (int m = 0; m < LB; ++m) lnx[m] = P.lu_l[min(i, n2 - 1) * kMaxBand + m];
    };
    load_l(0);
    auto step = [&](int i, double2 b) __attribute__((always_inline)) {
      double lc[LB];
#pragma unroll
      for (int m = 0; m < LB; ++m) lc[m] = lnx[m];
      load_l(i + 1);
#pragma unroll
      for (int m = 0; m < LB; ++m) b = fma2(-lc[m], ring[m], b);
      yp[size_t(i) * ncol + c] = b;
#pragma unroll
      for (int m = LB - 1; m > 0; --m) ring[m] = ring[m - 1];
      ring[0] = b;
    };
    double2 pf[kPreMc];  // slot d: the next row i = d (mod kPreMc)
#pragma unroll
    for (int d = 0; d < kPreMc; ++d) pf[d] = vals[size_t(min(d, n2 - 1)) * ncol + c];
    const int nfull = n2 - n2 % kPreMc;
    for (int i0 = 0; i0 < nfull; i0 += kPreMc) {
#pragma unroll
      for (int d = 0; d < kPreMc; ++d) {
        const int i = i0 + d;
        step(i, pf[d]);
        pf[d] = vals[size_t(min(i + kPreMc, n2 - 1)) * ncol + c];
      }
    }
#pragma unroll
    for (int d = 0; d < kPreMc; ++d)
      if (nfull + d < n2) step(nfull + d, pf[d]);
  }
  // 2. descending sweep: rho_t coefficients, r = -G1 rho_t, bottom-up forward sweep of A(k)
  {
    double* su = lds_d;                 // [n2][LB]
    double* sui = su + n2 * LB;         // [n2]
    double* sg = sui + n2;              // [N][kMaxW] G1 rows
    double* sds = sg + N * kMaxW;       // [n2] dstar
    int* sgc = reinterpret_cast<int*>(sds + n2);  // [n2] G1 emission counts
    int* snm = sgc + n2;                // [N]
    int* sof = snm + N;                 // [N]
    if constexpr (STAGE) {
      for (int e = threadIdx.x; e < n2 * LB; e += blockDim.x) su[e] = P.lu_u[(e / LB) * (kMaxBand + 1) + e % LB + 1];
      for (int e = threadIdx.x; e < n2; e += blockDim.x) {
        sui[e] = P.lu_uinv[e];
        sds[e] = P.dstar[e];
        sgc[e] = P.g1e_cnt[e];
      }
      for (int e = threadIdx.x; e < N * kMaxW; e += blockDim.x) sg[e] = P.gs_w[size_t(N) * kMaxW + e];
      for (int e = threadIdx.x; e < N; e += blockDim.x) {
        snm[e] = P.fac_nm[e];
        sof[e] = P.fac_off[e];
      }
      __syncthreads();
    }
    auto U_ = [&](int j, int q) -> double {
      if constexpr (STAGE) return su[j * LB + q]; else return P.lu_u[j * (kMaxBand + 1) + q + 1];
    };
    auto Ui_ = [&](int j) -> double { if constexpr (STAGE) return sui[j]; else return P.lu_uinv[j]; };
    auto G_ = [&](int i, int q) -> double {
      if constexpr (STAGE) return sg[i * kMaxW + q]; else return P.gs_w[(size_t(N) + i) * kMaxW + q];
    };
    auto ds_ = [&](int j) -> double { if constexpr (STAGE) return sds[j]; else return P.dstar[j]; };
    auto gc_ = [&](int j) -> int { if constexpr (STAGE) return sgc[j]; else return P.g1e_cnt[j]; };
    auto nm_ = [&](int r) -> int { if constexpr (STAGE) return snm[r]; else return P.fac_nm[r]; };
    auto of_ = [&](int r) -> int { if constexpr (STAGE) return sof[r]; else return P.fac_off[r]; };
    if (active) {
      double2 win[kMaxW];  // rho_t coefficients of rows j .. j+kMaxW-1
      double2 yr[UA];      // forward-sweep results of rows i+1 .. i+UA
#pragma unroll
      for (int q = 0; q < kMaxW; ++q) win[q] = zero2();
#pragma unroll
      for (int m = 0; m < UA; ++m) yr[m] = zero2();
      double2 cm = zero2();  // mean column: c_{j+1}
      yt[size_t(n2) * ncol + c] = zero2();  // Robin row n2: r = 0, nothing above it
      // multipliers of the next row of the bottom-up sweep (rows n2-1, n2-2, ..., 0 in turn), raw (the
      // entries past the row's count are masked where they are used): the rows are emitted a variable
      // number per step, so they are read one emission ahead, each row's as soon as the previous one's
      // have been used
      int inext = n2 - 1;
      double fm[UA];
      auto load_mult = [&](int row) __attribute__((always_inline)) {
        row = max(row, 0);
        const int nm = nm_(row), off = of_(row);
#pragma unroll
        for (int m = 0; m < UA; ++m) fm[m] = fac[(size_t(off) + min(m, max(nm - 1, 0))) * npairs];
      };
      auto mult = [&](int row, double2 r) __attribute__((always_inline)) {
        const int nm = nm_(row);
#pragma unroll
        for (int m = 0; m < UA; ++m) r = fma2(-(m < nm ? fm[m] : 0.0), yr[m], r);
        return r;
      };
      load_mult(inext);
      // the next step's U row, inverse pivot and emission count, and the G1 weights of the next row to
      // emit, are read while the current step (emission) runs: the table reads are not on the chain
      double nu[LB + 1], ng[kMaxW];
      int ncnt;
      auto load_row = [&](int j) __attribute__((always_inline)) {
        j = max(j, 0);
#pragma unroll
        for (int q = 0; q < LB; ++q) nu[q] = U_(j, q);
        nu[LB] = Ui_(j);
        ncnt = gc_(j);
      };
      auto load_g = [&](int i) __attribute__((always_inline)) {
        i = max(i, 0);
#pragma unroll
        for (int q = 0; q < kMaxW; ++q) ng[q] = G_(i, q);
      };
      load_row(n2 - 1);
      load_g(n2 - 1);
      auto step = [&](int j, double2 y) __attribute__((always_inline)) {
        double uc[LB + 1];
#pragma unroll
        for (int q = 0; q <= LB; ++q) uc[q] = nu[q];
        const int cnt = ncnt;
        load_row(j - 1);
#pragma unroll
        for (int q = 0; q < LB; ++q) y = fma2(-uc[q], win[q], y);
        const double2 x = cscale(y, uc[LB]);
#pragma unroll
        for (int q = kMaxW - 1; q > 0; --q) win[q] = win[q - 1];
        win[0] = x;
        if (rhoc) rhoc[size_t(j) * ncol + c] = x;
        if (mean) {
          cm = make_double2(cm.x + x.x / ds_(j), cm.y + x.y / ds_(j));
          yt[size_t(j) * ncol + c] = cm;
          return;
        }
        // rows are emitted in descending order, each once: the row is inext
        for (int e = 0; e < cnt; ++e) {
          const int i = inext;
          double gw[kMaxW];
#pragma unroll
          for (int q = 0; q < kMaxW; ++q) gw[q] = ng[q];
          load_g(i - 1);
          double2 r = zero2();
#pragma unroll
          for (int q = 0; q < kMaxW; ++q) r = fma2(-gw[q], win[q], r);
          r = mult(i, r);
          --inext;
          load_mult(inext);
          yt[size_t(i) * ncol + c] = r;
#pragma unroll
          for (int m = UA - 1; m > 0; --m) yr[m] = yr[m - 1];
          yr[0] = r;
        }
      };
      // step t of the sweep is row j = n2 - 1 - t of the L-sweep result; slot d serves t = d (mod kPreMc2)
      double2 pf[kPreMc2];
#pragma unroll
      for (int d = 0; d < kPreMc2; ++d) pf[d] = yp[size_t(max(n2 - 1 - d, 0)) * ncol + c];
      const int nfull = n2 - n2 % kPreMc2;
      for (int t0 = 0; t0 < nfull; t0 += kPreMc2) {
#pragma unroll
        for (int d = 0; d < kPreMc2; ++d) {
          const int j = n2 - 1 - (t0 + d);
          step(j, pf[d]);
          pf[d] = yp[size_t(max(j - kPreMc2, 0)) * ncol + c];
        }
      }
#pragma unroll
      for (int d = 0; d < kPreMc2; ++d)
        if (nfull + d < n2) step(n2 - 1 - (nfull + d), pf[d]);
      if (!mean) yt[c] = mult(0, zero2());  // Robin row 0 (inext == 0): r = 0
    }
  }
  // 3. ascending back substitution and emission of the values at tau
  {
    double* sw = lds_d;                  // [2][n2][kMaxW] F0, F1 emission weights
    double* sds = sw + 2 * n2 * kMaxW;   // [n2] dstar
    int* saf = reinterpret_cast<int*>(sds + n2);  // [N] emission starts
    int* sac = saf + N;                  // [N]
    int* snm = sac + N;                  // [N]
    int* sns = snm + N;                  // [N]
    int* sof = sns + N;                  // [N]
    if constexpr (STAGE) {
      __syncthreads();  // phase-2 tables no longer read
      for (int e = threadIdx.x; e < 2 * n2 * kMaxW; e += blockDim.x) sw[e] = P.asc_w[e];
      for (int e = threadIdx.x; e < n2; e += blockDim.x) sds[e] = P.dstar[e];
      for (int e = threadIdx.x; e < N; e += blockDim.x) {
        saf[e] = P.asc_first[e];
        sac[e] = P.asc_cnt[e];
        snm[e] = P.fac_nm[e];
        sns[e] = P.fac_ns[e];
        sof[e] = P.fac_off[e];
      }
      __syncthreads();
    }
    (void)lay;
    auto W_ = [&](int d, int row, int q) -> double {
      if constexpr (STAGE) return sw[(d * n2 + row) * kMaxW + q];
      else return P.asc_w[(size_t(d) * n2 + row) * kMaxW + q];
    };
    auto ds_ = [&](int j) -> double { if constexpr (STAGE) return sds[j]; else return P.dstar[j]; };
    auto af_ = [&](int j) -> int { if constexpr (STAGE) return saf[j]; else return P.asc_first[j]; };
    auto ac_ = [&](int j) -> int { if constexpr (STAGE) return sac[j]; else return P.asc_cnt[j]; };
    auto nm_ = [&](int r) -> int { if constexpr (STAGE) return snm[r]; else return P.fac_nm[r]; };
    auto ns_ = [&](int r) -> int { if constexpr (STAGE) return sns[r]; else return P.fac_ns[r]; };
    auto of_ = [&](int r) -> int { if constexpr (STAGE) return sof[r]; else return P.fac_off[r]; };
    if (active) {
      double2 cw[kMaxW];  // c_i, c_{i-1}, ...
#pragma unroll
      for (int q = 0; q < kMaxW; ++q) cw[q] = zero2();
      // entries left of the diagonal (raw[0 .. LA-1], those past the row's count masked at use) and
      // 1/pivot (raw[LA]) of a factor row, read unconditionally at an in-range address
      auto load_sub = [&](double (&dst)[LA + 1], int row) {
        row = min(row, N - 1);
        const int nm = nm_(row), ns = ns_(row), off = of_(row);
#pragma unroll
        for (int q = 0; q < LA; ++q) dst[q] = fac[(size_t(off) + nm + min(q, ns)) * npairs];
        dst[LA] = fac[(size_t(off) + nm + ns) * npairs];
      };
      // operands of the next tau row to emit (rows are emitted in ascending order, each once), read one
      // emission ahead: its input value and, for the final iterate, its m^d values
      double2 ev = vals[c], e1 = zero2(), e2 = zero2(), e3 = zero2();
      if (d1) {
        e1 = d1[c];
        e2 = d2[c];
        e3 = d3[c];
      }
      // rh: rho_t coefficient of row i - 1 (final iterate only), read with the step's other rows
      auto step = [&](int i, double2 x, const double (&fr)[LA + 1], double2 rh) __attribute__((always_inline)) {
        if (!mean) {
          const int ns = ns_(i);
#pragma unroll
          for (int q = 0; q < LA; ++q) x = fma2(-(q < ns ? fr[q] : 0.0), cw[q], x);
          x = cscale(x, fr[LA]);
        }
#pragma unroll
        for (int q = kMaxW - 1; q > 0; --q) cw[q] = cw[q - 1];
        cw[0] = x;
        if (c2) {
          c2[size_t(i) * ncol + c] = x;
          if (i > 0) {
            const size_t e = size_t(i - 1) * ncol + c;
            const double ds = ds_(i - 1);
            const double2 dc = make_double2(ds * (cw[0].x - cw[1].x), ds * (cw[0].y - cw[1].y));
            mparc[e] = mean ? zero2() : cscale(times_i(cadd(rh, dc)), ik);
          }
        }
        const int first = af_(i), cnt = ac_(i);
        for (int e = 0; e < cnt; ++e) {
          const int row = first + e;
          double2 m2 = zero2(), f1 = zero2();
#pragma unroll
          for (int q = 0; q < kMaxW; ++q) {
            m2 = fma2(W_(0, row, q), cw[q], m2);
            f1 = fma2(W_(1, row, q), cw[q], f1);
          }
          const size_t o = size_t(row) * ncol + c;
          double2 m1 = zero2(), m3 = zero2();
          if (!mean) {
            const double2 sum = cadd(ev, f1);  // rho_t + F1 c
            if (V3) {
              const double2 mp = cscale(times_i(sum), ik);
              m1 = cscale(mp, k1 * ik);
              m3 = cscale(mp, k3 * ik);
            } else {
              m1 = cscale(sum, ik * ik);  // psi: m1 = i k1 psi, m3 = i k3 psi
            }
          }
          if (d1) {
            m1 = cadd(m1, e1);
            m2 = cadd(m2, e2);
            m3 = cadd(m3, e3);
          }
          {  // the next emitted row is row + 1
            const size_t on = size_t(min(row + 1, n2 - 1)) * ncol + c;
            ev = vals[on];
            if (d1) {
              e1 = d1[on];
              e2 = d2[on];
              e3 = d3[on];
            }
          }
          V1[o] = m1;
          V2[o] = m2;
          if (V3) V3[o] = m3;
        }
      };
      // slot d serves rows i = d (mod kPreMc3): the A(k) forward-sweep result and the factor row
      double2 pf[kPreMc3], prh[kPreMc3];
      double fs[kPreMc3][LA + 1];
#pragma unroll
      for (int d = 0; d < kPreMc3; ++d) {
        pf[d] = yt[size_t(min(d, N - 1)) * ncol + c];
        load_sub(fs[d], d);
        prh[d] = c2 ? rhoc[size_t(max(d - 1, 0)) * ncol + c] : zero2();
      }
      const int nfull = N - N % kPreMc3;
      for (int i0 = 0; i0 < nfull; i0 += kPreMc3) {
#pragma unroll
        for (int d = 0; d < kPreMc3; ++d) {
          const int i = i0 + d;
          step(i, pf[d], fs[d], prh[d]);
          pf[d] = yt[size_t(min(i + kPreMc3, N - 1)) * ncol + c];
          load_sub(fs[d], i + kPreMc3);
          if (c2) prh[d] = rhoc[size_t(min(i + kPreMc3 - 1, n2 - 1)) * ncol + c];
        }
      }
#pragma unroll
      for (int d = 0; d < kPreMc3; ++d)
        if (nfull + d < N) step(nfull + d, pf[d], fs[d], prh[d]);
    }
  }
}
template <int LA, int UA, int LB, bool STAGE>
__global__ void __launch_bounds__(kThreads) k_mc(DevPlan P, const double2* __restrict__ vals, double2* yp, double2* yt,
                                  const double2* __restrict__ d1, const double2* __restrict__ d2,
                                  const double2* __restrict__ d3, double2* __restrict__ V1, double2* __restrict__ V2,
                                  double2* __restrict__ V3, double2* rhoc, double2* __restrict__ c2,
                                  double2* __restrict__ mparc) {
  mc_body<LA, UA, LB, STAGE>(P, blockIdx.x, vals, yp, yt, d1, d2, d3, V1, V2, V3, rhoc, c2, mparc);
}

// ---------------------------------------------------------------------------
// column kernel: m^d and its values at tau (eqs. phi_poisson, bc_both,
// md_recon), one thread per column, pairs (l, +-n) on neighbouring lanes.
//   1. descending sweep: r_i = G0 phi2 at the interior tau* rows (phi2 read
//      through a register window of W = p rows, every coefficient once),
//      bottom-up forward sweep of A(k) c = r (per-plan factors, Robin rows r = 0);
//   2. ascending back substitution for c (B* coefficients of m2); every tau
//      row whose F0/F1 band is complete emits
//        m2 = F0 c,  m1 = (i k1 F1 c - i k3 E0 Omega2)/k^2,  m3 = (i k3 F1 c + i k1 E0 Omega2)/k^2
//      (F1 = E0 D*, Omega2 read through a second window).
// Plane mean: m^d = (<m>1, 0, <m>3).  With c2o the coefficients are written too.
struct MdArgs {
  const double2 *phi, *om;
  const double *m1bar, *m3bar;
  double2 *yt, *V1, *V2, *V3, *c2o, *m1o, *m3o;
};
template <int LA, int UA, int W>
__device__ __forceinline__ void md_body(const DevPlan& P, int t, const MdArgs& A) {
  const double2* __restrict__ phi = A.phi;
  const double2* __restrict__ om = A.om;
  const double* __restrict__ m1bar = A.m1bar;
  const double* __restrict__ m3bar = A.m3bar;
  double2* yt = A.yt;
  double2* __restrict__ V1 = A.V1;
  double2* __restrict__ V2 = A.V2;
  double2* __restrict__ V3 = A.V3;
  double2* __restrict__ c2o = A.c2o;
  double2* __restrict__ m1o = A.m1o;
  double2* __restrict__ m3o = A.m3o;
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const int half = (nn + 1) / 2, npairs = nl * half;
  const int pr = t >> 1, side = t & 1;
  if (pr >= npairs) return;
  const int l = pr % nl, pp = pr / nl;
  if (side == 1 && pp == 0) return;
  const int ni = side ? nn - pp : pp;
  const size_t ncol = size_t(nn) * nl, c = size_t(ni) * nl + l;
  const double k1 = P.k1[l], k3 = P.k3[ni], ksq = k1 * k1 + k3 * k3;
  if (ksq == 0.0) {
    for (int i = 0; i < n2; ++i) {
      const int lo = P.ev_lo[i];
      double a1 = 0.0, a3 = 0.0;
      for (int q = 0; q < kMaxW; ++q)
        if (lo + q < n2) {
          a1 += P.ev_w[size_t(i) * kMaxW + q] * m1bar[lo + q];
          a3 += P.ev_w[size_t(i) * kMaxW + q] * m3bar[lo + q];
        }
      V1[size_t(i) * ncol] = make_double2(a1, 0.0);
      V2[size_t(i) * ncol] = zero2();
      V3[size_t(i) * ncol] = make_double2(a3, 0.0);
    }
    if (c2o) {
      for (int i = 0; i < N; ++i) c2o[size_t(i) * ncol] = zero2();
      for (int i = 0; i < n2; ++i) {
        m1o[size_t(i) * ncol] = make_double2(m1bar[i], 0.0);
        m3o[size_t(i) * ncol] = make_double2(m3bar[i], 0.0);
      }
    }
    return;
  }
  const double iksq = 1.0 / ksq;
  const double* fac = P.fac + pr;
  // 1. descending: r = G0 phi2, bottom-up forward sweep
  {
    double2 wp[W];  // phi2 rows base .. base+W-1
    int base = n2 - W;
#pragma unroll
    for (int q = 0; q < W; ++q) wp[q] = phi[size_t(base + q) * ncol + c];
    double2 yr[UA];
#pragma unroll
    for (int m = 0; m < UA; ++m) yr[m] = zero2();
    double fm[UA];
    auto load_mult = [&](int row) {
      const int nm = P.fac_nm[row], off = P.fac_off[row];
#pragma unroll
      for (int m = 0; m < UA; ++m) fm[m] = (m < nm) ? fac[(size_t(off) + m) * npairs] : 0.0;
    };
    yt[size_t(n2) * ncol + c] = zero2();  // Robin row n2: r = 0
    load_mult(n2 - 1);
    for (int i = n2 - 1; i >= 1; --i) {
      const int lo = P.gs_lo[i];
      while (base > lo) {
#pragma unroll
        for (int q = W - 1; q > 0; --q) wp[q] = wp[q - 1];
        --base;
        wp[0] = phi[size_t(base) * ncol + c];
      }
      double2 r = zero2();
#pragma unroll
      for (int q = 0; q < W; ++q) r = fma2(P.gs_w[size_t(i) * kMaxW + q], wp[q], r);
#pragma unroll
      for (int m = 0; m < UA; ++m) r = fma2(-fm[m], yr[m], r);
      load_mult(i - 1);
      yt[size_t(i) * ncol + c] = r;
#pragma unroll
      for (int m = UA - 1; m > 0; --m) yr[m] = yr[m - 1];
      yr[0] = r;
    }
    double2 r = zero2();  // Robin row 0
#pragma unroll
    for (int m = 0; m < UA; ++m) r = fma2(-fm[m], yr[m], r);
    yt[c] = r;
  }
  // 2. ascending back substitution, emission of the values at tau
  {
    double2 cw[kMaxW];
#pragma unroll
    for (int q = 0; q < kMaxW; ++q) cw[q] = zero2();
    RowWin<W> wo;
    wo.init(om, ncol, c, n2);
    double fs[LA + 1];
    auto load_sub = [&](int row) {
      const int nm = P.fac_nm[row], ns = P.fac_ns[row], off = P.fac_off[row];
#pragma unroll
      for (int q = 0; q < LA; ++q) fs[q] = (q < ns) ? fac[(size_t(off) + nm + q) * npairs] : 0.0;
      fs[LA] = fac[(size_t(off) + nm + ns) * npairs];
    };
    double2 ytn = yt[c];
    load_sub(0);
    for (int i = 0; i < N; ++i) {
      double2 x = ytn;
      double fc[LA + 1];
#pragma unroll
      for (int q = 0; q <= LA; ++q) fc[q] = fs[q];
      if (i + 1 < N) {
        ytn = yt[size_t(i + 1) * ncol + c];
        load_sub(i + 1);
      }
#pragma unroll
      for (int q = 0; q < LA; ++q) x = fma2(-fc[q], cw[q], x);
      x = cscale(x, fc[LA]);
#pragma unroll
      for (int q = kMaxW - 1; q > 0; --q) cw[q] = cw[q - 1];
      cw[0] = x;
      if (c2o) {
        c2o[size_t(i) * ncol + c] = x;
        if (i > 0) {
          const size_t e = size_t(i - 1) * ncol + c;
          const double ds = P.dstar[i - 1];
          const double2 D = make_double2(ds * (cw[0].x - cw[1].x), ds * (cw[0].y - cw[1].y));
          const double2 O = om[e];
          m1o[e] = cscale(times_i(make_double2(k1 * D.x - k3 * O.x, k1 * D.y - k3 * O.y)), iksq);
          m3o[e] = cscale(times_i(make_double2(k3 * D.x + k1 * O.x, k3 * D.y + k1 * O.y)), iksq);
        }
      }
      const int first = P.asc_first[i], cnt = P.asc_cnt[i];
      for (int e = 0; e < cnt; ++e) {
        const int row = first + e;
        double2 f0 = zero2(), f1 = zero2();
#pragma unroll
        for (int q = 0; q < kMaxW; ++q) {
          f0 = fma2(P.asc_w[size_t(row) * kMaxW + q], cw[q], f0);
          f1 = fma2(P.asc_w[(size_t(n2) + row) * kMaxW + q], cw[q], f1);
        }
        wo.advance(om, ncol, c, n2, P.ev_lo[row]);
        const double2 oe = wo.dot(P.ev_w + size_t(row) * kMaxW);
        const size_t o = size_t(row) * ncol + c;
        V1[o] = cscale(times_i(make_double2(k1 * f1.x - k3 * oe.x, k1 * f1.y - k3 * oe.y)), iksq);
        V2[o] = f0;
        V3[o] = cscale(times_i(make_double2(k3 * f1.x + k1 * oe.x, k3 * f1.y + k1 * oe.y)), iksq);
      }
    }
  }
}

// The substep's first column work in one launch, one job per blockIdx.y (the
// jobs are independent; together they fill the GPU better than one by one):
// job 0 m^d and its values (only when `md` is set), then the values of z and
// the BDF-like guess.
template <int LA, int UA, int W>
__global__ void __launch_bounds__(kThreads) k_prologue(DevPlan P, int md, MdArgs M, ValuesZArgs Z, GuessArgs G) {
  const int job = int(blockIdx.y) + (md ? 0 : 1);
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (job == 0) md_body<LA, UA, W>(P, int(t), M);
  else if (job == 1) values_z_body(P, t, Z);
  else guess_body(P, t, G);
}

// ---------------------------------------------------------------------------
// column kernel: the right-hand sides of Omega2 and phi2 at tau (from the
// flux kernels) -> coefficients with Dirichlet end rows, RK2 update.

__device__ __forceinline__ void rhs_fluct_body(const DevPlan& P, const unsigned bx, const double2* __restrict__ RO,
                                               const double2* __restrict__ RP, const double2* phi, const double2* om,
                                               const double2* __restrict__ rphi_prev,
                                               const double2* __restrict__ rom_prev, double2* phi_out, double2* om_out,
                                               double2* __restrict__ rphi_out, double2* __restrict__ rom_out,
                                               double2* __restrict__ yphi, double2* __restrict__ yom, int stage) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2;
  const int ncol = nn * nl;
  const int c = bx * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  (void)nl;
  const auto L = P.lu_l + size_t(1) * n2 * kMaxBand;
  const auto U = P.lu_u + size_t(1) * n2 * (kMaxBand + 1);
  const auto Ui = P.lu_uinv + size_t(1) * n2;
  constexpr int D = kProjPre;
  const int nfull = n2 - n2 % D;
  double2 rp[kMaxBand], ro[kMaxBand];
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) rp[m] = ro[m] = zero2();
  // ascending L sweep over the interior rows (Dirichlet end rows zero); rows come through rings of D
  // slots, slot d serving the steps i = d (mod D), each consumed before its refill is issued
  // the band row of the next step is read while the current step runs (scalar loads, one row ahead)
  double lnx[kMaxBand];
  auto load_l = [&](int i) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) lnx[m] = L[min(i, n2 - 1) * kMaxBand + m];
  };
  auto fwd = [&](int i, double2 bp, double2 bo) __attribute__((always_inline)) {
    double lc[kMaxBand];
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) lc[m] = lnx[m];
    load_l(i + 1);
    if (i == 0 || i == n2 - 1) bp = bo = zero2();
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) {
      bp = fma2(-lc[m], rp[m], bp);
      bo = fma2(-lc[m], ro[m], bo);
    }
    yphi[size_t(i) * ncol + c] = bp;
    yom[size_t(i) * ncol + c] = bo;
#pragma unroll
    for (int m = kMaxBand - 1; m > 0; --m) {
      rp[m] = rp[m - 1];
      ro[m] = ro[m - 1];
    }
    rp[0] = bp;
    ro[0] = bo;
  };
  {
    load_l(0);
    double2 pp[D], po[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      pp[d] = RP[size_t(min(d, n2 - 1)) * ncol + c];
      po[d] = RO[size_t(min(d, n2 - 1)) * ncol + c];
    }
    for (int i0 = 0; i0 < nfull; i0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = i0 + d;
        fwd(i, pp[d], po[d]);
        pp[d] = RP[size_t(min(i + D, n2 - 1)) * ncol + c];
        po[d] = RO[size_t(min(i + D, n2 - 1)) * ncol + c];
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (nfull + d < n2) fwd(nfull + d, pp[d], po[d]);
  }
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) rp[m] = ro[m] = zero2();
  // descending U sweep and the RK2 update; the state and the previous stage's right-hand sides are
  // read unconditionally (from the state itself when the stage does not use them)
  const bool upd = stage <= 1;
  const double2* phr = upd ? phi : yphi;
  const double2* omr = upd ? om : yom;
  const double2* ppr = stage == 1 ? rphi_prev : phr;
  const double2* opr = stage == 1 ? rom_prev : omr;
  struct Rows {
    double2 yp, yo, p0, o0, pp, op;
  };
  auto load = [&](Rows& r, int i) __attribute__((always_inline)) {
    const size_t e = size_t(i) * ncol + c;
    r.yp = yphi[e];
    r.yo = yom[e];
    r.p0 = phr[e];
    r.o0 = omr[e];
    r.pp = ppr[e];
    r.op = opr[e];
  };
  double unx[kMaxBand + 1];  // U row and inverse pivot of the next step, one row ahead
  auto load_u = [&](int i) __attribute__((always_inline)) {
    i = max(i, 0);
#pragma unroll
    for (int q = 0; q < kMaxBand; ++q) unx[q] = U[i * (kMaxBand + 1) + q + 1];
    unx[kMaxBand] = Ui[i];
  };
  auto bwd = [&](int i, const Rows& r) __attribute__((always_inline)) {
    const size_t e = size_t(i) * ncol + c;
    double uc[kMaxBand + 1];
#pragma unroll
    for (int q = 0; q <= kMaxBand; ++q) uc[q] = unx[q];
    load_u(i - 1);
    double2 yp = r.yp, yo = r.yo;
#pragma unroll
    for (int q = 0; q < kMaxBand; ++q) {
      yp = fma2(-uc[q], rp[q], yp);
      yo = fma2(-uc[q], ro[q], yo);
    }
    const double2 xp = cscale(yp, uc[kMaxBand]), xo = cscale(yo, uc[kMaxBand]);
#pragma unroll
    for (int q = kMaxBand - 1; q > 0; --q) {
      rp[q] = rp[q - 1];
      ro[q] = ro[q - 1];
    }
    rp[0] = xp;
    ro[0] = xo;
    if (rphi_out) rphi_out[e] = xp;
    if (rom_out) rom_out[e] = xo;
    if (!upd) return;  // right-hand sides only
    if (stage == 0) {
      phi_out[e] = fma2(0.5 * P.dt, xp, r.p0);
      om_out[e] = fma2(0.5 * P.dt, xo, r.o0);
    } else {
      phi_out[e] = fma2(P.dt, make_double2(xp.x - 0.5 * r.pp.x, xp.y - 0.5 * r.pp.y), r.p0);
      om_out[e] = fma2(P.dt, make_double2(xo.x - 0.5 * r.op.x, xo.y - 0.5 * r.op.y), r.o0);
    }
  };
  {
    load_u(n2 - 1);
    Rows pr[D];  // slot d: step t = d (mod D), row i = n2 - 1 - t
#pragma unroll
    for (int d = 0; d < D; ++d) load(pr[d], max(n2 - 1 - d, 0));
    for (int t0 = 0; t0 < nfull; t0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int i = n2 - 1 - (t0 + d);
        bwd(i, pr[d]);
        load(pr[d], max(i - D, 0));
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (nfull + d < n2) bwd(n2 - 1 - (nfull + d), pr[d]);
  }
}
__global__ void __launch_bounds__(kThreads) k_rhs_fluct(DevPlan P, const double2* __restrict__ RO,
                                  const double2* __restrict__ RP, const double2* phi, const double2* om,
                                  const double2* __restrict__ rphi_prev, const double2* __restrict__ rom_prev,
                                  double2* phi_out, double2* om_out, double2* __restrict__ rphi_out,
                                  double2* __restrict__ rom_out, double2* __restrict__ yphi, double2* __restrict__ yom,
                                  int stage) {
  rhs_fluct_body(P, blockIdx.x, RO, RP, phi, om, rphi_prev, rom_prev, phi_out, om_out, rphi_out, rom_out, yphi, yom,
                 stage);
}

// plane means <m>1, <m>3: RHS = d/dy <T12>, d/dy <T32> at tau, Neumann rows,
// RK2 (eq. mean_m1m3).
__device__ __forceinline__ void rhs_mean_body(const DevPlan& P, const unsigned bx, const double2* __restrict__ T12,
                                              const double2* __restrict__ T23, const double* m1, const double* m3,
                                              const double* __restrict__ r1p, const double* __restrict__ r3p,
                                              double* m1o, double* m3o, double* __restrict__ r1o,
                                              double* __restrict__ r3o, int stage) {
  // one block: the right-hand sides of both components, all rows in parallel,
  // then one thread per component runs the two sweeps with the band in
  // registers (the rows are a dependent chain), then the updates in parallel
  extern __shared__ double ysh[];  // [2][n2]
  const int n2 = P.n2;
  const size_t ncol = size_t(P.nn) * P.nl;
  for (int t = threadIdx.x; t < 2 * n2; t += blockDim.x) {
    const int comp = t / n2, i = t - comp * n2;
    const double2* T = comp == 0 ? T12 : T23;
    double b = 0.0;
    if (i > 0 && i < n2 - 1) {
      const int lo = P.ev_lo[n2 + i];
      const auto w1 = P.ev_w + (size_t(1) * n2 + i) * kMaxW;
      for (int q = 0; q < kMaxW; ++q)
        if (lo + q < n2 && w1[q] != 0.0) b += w1[q] * T[size_t(lo + q) * ncol].x;
    }
    ysh[t] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double* y = ysh + threadIdx.x * n2;
    const auto L = P.lu_l + size_t(2) * n2 * kMaxBand;
    const auto U = P.lu_u + size_t(2) * n2 * (kMaxBand + 1);
    const auto Ui = P.lu_uinv + size_t(2) * n2;
    double ring[kMaxBand];
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) ring[m] = 0.0;
    for (int i = 0; i < n2; ++i) {  // L (unit lower, zero-padded band): ring[m] = y[i-1-m]
      double b = y[i];
#pragma unroll
      for (int m = 0; m < kMaxBand; ++m) b -= L[i * kMaxBand + m] * ring[m];
#pragma unroll
      for (int m = kMaxBand - 1; m > 0; --m) ring[m] = ring[m - 1];
      ring[0] = b;
      y[i] = b;
    }
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) ring[m] = 0.0;
    for (int i = n2 - 1; i >= 0; --i) {  // U: ring[q] = x[i+1+q]
      double v = y[i];
#pragma unroll
      for (int q = 0; q < kMaxBand; ++q) v -= U[i * (kMaxBand + 1) + q + 1] * ring[q];
      const double x = v * Ui[i];
#pragma unroll
      for (int q = kMaxBand - 1; q > 0; --q) ring[q] = ring[q - 1];
      ring[0] = x;
      y[i] = x;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 2 * n2; t += blockDim.x) {
    const int comp = t / n2, i = t - comp * n2;
    const double x = ysh[t];
    double* ro = comp == 0 ? r1o : r3o;
    const double* m = comp == 0 ? m1 : m3;
    const double* rprev = comp == 0 ? r1p : r3p;
    double* mo = comp == 0 ? m1o : m3o;
    if (ro) ro[i] = x;
    if (stage <= 1) mo[i] = (stage == 0) ? m[i] + 0.5 * P.dt * x : m[i] + P.dt * (x - 0.5 * rprev[i]);
  }
}
__global__ void __launch_bounds__(256) k_rhs_mean(DevPlan P, const double2* __restrict__ T12,
                                  const double2* __restrict__ T23, const double* m1, const double* m3,
                                  const double* __restrict__ r1p, const double* __restrict__ r3p, double* m1o,
                                  double* m3o, double* __restrict__ r1o, double* __restrict__ r3o, int stage) {
  rhs_mean_body(P, blockIdx.x, T12, T23, m1, m3, r1p, r3p, m1o, m3o, r1o, r3o, stage);
}

// ---------------------------------------------------------------------------
// Column kernels as jobs: an argument struct, the body on one instance (its
// plan, block index and arguments), the named single-instance launch, and one
// grouped kernel per job that runs the job for many instances (each its own
// plan and sizes) in a single launch: instance r owns blocks b0 .. b0+nbx-1.

template <class A>
struct GRec {
  A a;
  int inst;
  unsigned b0, nbx, nby;  // first block, and the x and y extents of the instance's grid
};

template <class Job>
__device__ __forceinline__ void group_dispatch(const DevPlan* __restrict__ plans,
                                               const GRec<typename Job::Args>* __restrict__ recs, int nrec) {
  const unsigned bid = blockIdx.x;
  int lo = 0, hi = nrec - 1;  // the last record with b0 <= bid (records ascend, no gaps)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (recs[mid].b0 <= bid) lo = mid;
    else hi = mid - 1;
  }
  const GRec<typename Job::Args>& R = recs[lo];
  const unsigned loc = bid - R.b0, rest = loc / R.nbx;
  Job::run(plans[R.inst], loc % R.nbx, rest % R.nby, rest / R.nby, R.a);
}
// one grouped kernel per job, with the job's own launch bounds
template <class Job>
__global__ void __launch_bounds__(Job::kBound) k_group(const DevPlan* __restrict__ plans,
                                                       const GRec<typename Job::Args>* __restrict__ recs, int nrec) {
  group_dispatch<Job>(plans, recs, nrec);
}
template <class Job>
__global__ void __launch_bounds__(Job::kBound, Job::kMinBlocks) k_group_mb(
    const DevPlan* __restrict__ plans, const GRec<typename Job::Args>* __restrict__ recs, int nrec) {
  group_dispatch<Job>(plans, recs, nrec);
}

// column jobs: 256-thread blocks
struct ColumnJob {
  static constexpr int kBound = kThreads, kBlock = kThreads, kMinBlocks = 0;
};

template <int LA, int UA, int W>
struct JobPrologue : ColumnJob {
  struct Args {
    int md;
    MdArgs M;
    ValuesZArgs Z;
    GuessArgs G;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& A) {
    const int job = int(by) + (A.md ? 0 : 1);
    const size_t t = size_t(bx) * blockDim.x + threadIdx.x;
    if (job == 0) md_body<LA, UA, W>(P, int(t), A.M);
    else if (job == 1) values_z_body(P, t, A.Z);
    else guess_body(P, t, A.G);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL((k_prologue<LA, UA, W>), g, dim3(kThreads), lds, s, P, A.md, A.M, A.Z, A.G);
  }
};

template <int EPI>
struct JobProj : ColumnJob {
  struct Args {
    int kind;
    const double2* in;
    double2* out;
    const double2 *add, *z, *zt_prev;
    double2 *z_out, *vals_out, *vals_out1;
    int stage, ncol;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    proj_body<EPI>(P, int(bx * blockDim.x + threadIdx.x), A.kind, A.in, A.out, A.add, A.z, A.zt_prev, A.z_out,
                   A.vals_out, A.vals_out1, A.stage, A.ncol);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL(k_proj<EPI>, g, dim3(kThreads), lds, s, P, A.kind, A.in, A.out, A.add, A.z, A.zt_prev,
                       A.z_out, A.vals_out, A.vals_out1, A.stage, A.ncol);
  }
};

struct JobProj3 : ColumnJob {
  struct Args {
    int kind;
    ProjBatch B;
    int ncol;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& A) {
    proj_body<EPI_STORE>(P, int(bx * blockDim.x + threadIdx.x), A.kind, A.B.in[by], A.B.out[by], nullptr, nullptr,
                         nullptr, nullptr, nullptr, nullptr, 0, A.ncol);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL(k_proj3, g, dim3(kThreads), lds, s, P, A.kind, A.B, A.ncol);
  }
};

template <int LA, int UA, int LB, bool STAGE>
struct JobMc : ColumnJob {
  struct Args {
    const double2* vals;
    double2 *yp, *yt;
    const double2 *d1, *d2, *d3;
    double2 *V1, *V2, *V3, *rhoc, *c2, *mparc;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    mc_body<LA, UA, LB, STAGE>(P, bx, A.vals, A.yp, A.yt, A.d1, A.d2, A.d3, A.V1, A.V2, A.V3, A.rhoc, A.c2,
                               A.mparc);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL((k_mc<LA, UA, LB, STAGE>), g, dim3(kThreads), lds, s, P, A.vals, A.yp, A.yt, A.d1, A.d2,
                       A.d3, A.V1, A.V2, A.V3, A.rhoc, A.c2, A.mparc);
  }
};

struct FluxArgs {
  const double2 *Ca, *Cb, *Cc, *u1, *u2, *u3;
  double2 *Ta, *Tb, *Tc, *RO, *RP;
  const double2* rhov;
};
template <int GROUP, int W, int LB, bool VARMU = false>
struct JobFlux : ColumnJob {
  using Args = FluxArgs;
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    flux_body<GROUP, W, LB, VARMU>(P, bx, A.Ca, A.Cb, A.Cc, A.u1, A.u2, A.u3, A.Ta, A.Tb, A.Tc, A.RO, A.RP,
                                   A.rhov);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL((k_flux<GROUP, W, LB, VARMU>), g, dim3(kThreads), lds, s, P, A.Ca, A.Cb, A.Cc, A.u1, A.u2, A.u3,
                       A.Ta, A.Tb, A.Tc, A.RO, A.RP, A.rhov);
  }
};

template <int W>
struct JobStrain : ColumnJob {
  struct Args {
    const double2 *u1, *u2, *u3;
    SixPtr S;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    strain_body<W>(P, bx, A.u1, A.u2, A.u3, A.S);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL((k_strain<W>), g, dim3(kThreads), lds, s, P, A.u1, A.u2, A.u3, A.S);
  }
};

struct JobRhsFluct : ColumnJob {
  struct Args {
    const double2 *RO, *RP, *phi, *om, *rphi_prev, *rom_prev;
    double2 *phi_out, *om_out, *rphi_out, *rom_out, *yphi, *yom;
    int stage;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    rhs_fluct_body(P, bx, A.RO, A.RP, A.phi, A.om, A.rphi_prev, A.rom_prev, A.phi_out, A.om_out, A.rphi_out,
                   A.rom_out, A.yphi, A.yom, A.stage);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL(k_rhs_fluct, g, dim3(kThreads), lds, s, P, A.RO, A.RP, A.phi, A.om, A.rphi_prev,
                       A.rom_prev, A.phi_out, A.om_out, A.rphi_out, A.rom_out, A.yphi, A.yom, A.stage);
  }
};

struct JobRhsMean : ColumnJob {
  struct Args {
    const double2 *T12, *T23;
    const double *m1, *m3, *r1p, *r3p;
    double *m1o, *m3o, *r1o, *r3o;
    int stage;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& A) {
    rhs_mean_body(P, bx, A.T12, A.T23, A.m1, A.m3, A.r1p, A.r3p, A.m1o, A.m3o, A.r1o, A.r3o, A.stage);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& A) {
    hipLaunchKernelGGL(k_rhs_mean, g, dim3(kThreads), lds, s, P, A.T12, A.T23, A.m1, A.m3, A.r1p, A.r3p, A.m1o,
                       A.m3o, A.r1o, A.r3o, A.stage);
  }
};

// plane jobs (register-FFT kernels; block shape fixed by the transform size)
template <int N, bool EXACT, int D = 1>
struct JobZinvR {
  static constexpr int kBound = kThreads, kBlock = ZShape<N, D>::LG * ZShape<N, D>::T, kMinBlocks = 0;
  struct Args {
    EvalArgs A;
    double2* zbuf;
    int j0, pb;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned bz, const Args& a) {
    zinv_r_body<N, EXACT, D>(P, bx, by, bz, a.A, a.zbuf, a.j0, a.pb);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL((k_zinv_r<N, EXACT, D>), g, dim3(kBlock), lds, s, P, a.A, a.zbuf, a.j0, a.pb);
  }
};
template <int N, int D = 1>
struct JobZfwdR {
  static constexpr int kBound = kThreads, kBlock = ZShape<N, D>::LG * ZShape<N, D>::T, kMinBlocks = 0;
  struct Args {
    const double2* obuf;
    OutPtrs V;
    int j0, pb;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned bz, const Args& a) {
    zfwd_r_body<N, D>(P, bx, by, bz, a.obuf, a.V, a.j0, a.pb);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL((k_zfwd_r<N, D>), g, dim3(kBlock), lds, s, P, a.obuf, a.V, a.j0, a.pb);
  }
};
template <int N, bool EXACT>
struct JobZinvW {
  static constexpr int kBound = kZWThreads, kBlock = kZWThreads, kMinBlocks = 0;
  using Args = typename JobZinvR<N, EXACT>::Args;
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned bz, const Args& a) {
    zinv_w_body<N, EXACT>(P, bx, by, bz, a.A, a.zbuf, a.j0, a.pb);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL((k_zinv_w<N, EXACT>), g, dim3(kBlock), lds, s, P, a.A, a.zbuf, a.j0, a.pb);
  }
};
template <int N>
struct JobZfwdW {
  static constexpr int kBound = kZWThreads, kBlock = kZWThreads, kMinBlocks = 0;
  using Args = typename JobZfwdR<N>::Args;
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned bz, const Args& a) {
    zfwd_w_body<N>(P, bx, by, bz, a.obuf, a.V, a.j0, a.pb);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL(k_zfwd_w<N>, g, dim3(kBlock), lds, s, P, a.obuf, a.V, a.j0, a.pb);
  }
};
template <int PH, int N>
struct JobXline {
  static constexpr int kBound = kThreads, kBlock = XPlan<N>::BG * XPlan<N>::T, kMinBlocks = 0;
  struct Args {
    const double2* zbuf;
    double2* obuf;
    int pb, j0;
    const double* aux;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& a) {
    xline_body<PH, N>(P, bx, by, a.zbuf, a.obuf, a.pb, a.j0, a.aux);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL((k_xline<PH, N>), g, dim3(kBlock), lds, s, P, a.zbuf, a.obuf, a.pb, a.j0, a.aux);
  }
};
template <int PH, int N, int MINB>
struct JobXpair {
  static constexpr int kBound = kThreads, kBlock = XPlan<N>::BG * XPlan<N>::T, kMinBlocks = MINB;
  struct Args {
    const double2* zbuf;
    double2* obuf;
    int pb;
    double* phys_out;
    const double* phys_in;
    int j0;
    double* aux;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& a) {
    xpair_body<PH, N>(P, bx, by, a.zbuf, a.obuf, a.pb, a.phys_out, a.phys_in, a.j0, a.aux);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    if constexpr (MINB == 2)
      hipLaunchKernelGGL((k_xpair_w2<PH, N>), g, dim3(kBlock), lds, s, P, a.zbuf, a.obuf, a.pb, a.phys_out,
                         a.phys_in, a.j0, a.aux);
    else
      hipLaunchKernelGGL((k_xpair<PH, N>), g, dim3(kBlock), lds, s, P, a.zbuf, a.obuf, a.pb, a.phys_out, a.phys_in,
                         a.j0, a.aux);
  }
};

template <int N>
struct JobZfiltW {
  static constexpr int kBound = kZWThreads, kBlock = kZWThreads, kMinBlocks = 0;
  struct Args {
    const double2 *in, *add;
    double2* out;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& a) {
    zfilt_w_body<N>(P, bx, by, a.in, a.add, a.out);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL(k_zfilt_w<N>, g, dim3(kBlock), lds, s, P, a.in, a.add, a.out);
  }
};
template <int N, int D = 1>
struct JobZfiltR {
  static constexpr int kBound = kThreads, kBlock = ZShape<N, D>::LG * ZShape<N, D>::T, kMinBlocks = 0;
  using Args = typename JobZfiltW<N>::Args;
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned by, unsigned, const Args& a) {
    zfilt_r_body<N, D>(P, bx, by, a.in, a.add, a.out);
  }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL((k_zfilt_r<N, D>), g, dim3(kBlock), lds, s, P, a.in, a.add, a.out);
  }
};
struct JobWall : ColumnJob {
  struct Args {
    double2* zt;
  };
  __device__ static void run(const DevPlan& P, unsigned bx, unsigned, unsigned, const Args& a) { wall_body(P, bx, a.zt); }
  static void launch(dim3 g, size_t lds, hipStream_t s, const DevPlan& P, const Args& a) {
    hipLaunchKernelGGL(k_wall, g, dim3(kThreads), lds, s, P, a.zt);
  }
};

// BDF-like guess dt z_t^0 = a1 z + a2 h1 + a3 h2 + a4 h3 (eq. dzdt_guesses)
__global__ void k_guess(const double2* __restrict__ z, const double2* __restrict__ h1, const double2* __restrict__ h2,
                        const double2* __restrict__ h3, double a1, double a2, double a3, double a4, double dt,
                        double2* __restrict__ out, size_t n, int zero) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (zero) {
    out[e] = zero2();
    return;
  }
  const double2 a = z[e], b = h1[e], c = h2[e], d = h3[e];
  out[e] = make_double2((a1 * a.x + a2 * b.x + a3 * c.x + a4 * d.x) / dt,
                        (a1 * a.y + a2 * b.y + a3 * c.y + a4 * d.y) / dt);
}

// z update from a given z_t (used when k_f = 0)
__global__ void k_zupdate(const double2* __restrict__ z, const double2* __restrict__ zt,
                          const double2* __restrict__ ztp, double2* __restrict__ zo, double dt, int stage, size_t n) {
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 a = z[e], t = zt[e];
  if (stage == 0) {
    zo[e] = make_double2(a.x + 0.5 * dt * t.x, a.y + 0.5 * dt * t.y);
  } else {
    const double2 p = ztp[e];
    zo[e] = make_double2(a.x + dt * (t.x - 0.5 * p.x), a.y + dt * (t.y - 0.5 * p.y));
  }
}

// plain evaluation (operator entry point)
__global__ void k_evaluate(DevPlan P, int kind, const double2* __restrict__ src, double2* __restrict__ dst) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ncol * P.n2) return;
  const int j = int(e / ncol);
  const size_t col = e - size_t(j) * ncol;
  dst[e] = eval_at(P, kind, src, j, col, ncol, 0.0);
}

// ---------------------------------------------------------------------------
// adjoints (transposes in the real inner products <a, b> = sum Re(conj(a) b) of S-fields and
// sum f g of physical fields) of evaluation, projection and the inverse transform

// E_d^T: values at tau (n2 rows) -> coefficients (n2 rows, n2 + 1 for F0), one thread per (coefficient row,
// column), grid (ceil(ncol / 256), rows).  Coefficient row i gathers the value rows j whose band
// [lo_j, lo_j + kMaxW) holds it; lo_j is nondecreasing, so they are one range [ja, jb], found by binary
// search on the (uniform) row table, and summed in ascending j.
__global__ void __launch_bounds__(kThreads) k_evaluate_t(DevPlan P, int kind, const double2* __restrict__ src,
                                                        double2* __restrict__ dst) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int i = int(blockIdx.y);
  const int n2 = P.n2, rows = (kind == EV_F0) ? n2 + 1 : n2;
  if (c >= ncol || i >= rows) return;
  const cptr<int> lo = P.ev_lo + size_t(kind) * n2;
  // ja: first j with lo_j + kMaxW - 1 >= i;  jb: last j with lo_j <= i
  int a0 = 0, a1 = n2;
  while (a0 < a1) {
    const int m = (a0 + a1) >> 1;
    if (lo[m] + kMaxW - 1 < i) a0 = m + 1; else a1 = m;
  }
  int b0 = a0, b1 = n2;
  while (b0 < b1) {
    const int m = (b0 + b1) >> 1;
    if (lo[m] <= i) b0 = m + 1; else b1 = m;
  }
  double2 acc = zero2();
  for (int j = a0; j < b0; ++j) {
    const int q = i - lo[j];
    acc = fma2(P.ev_w[(size_t(kind) * n2 + j) * kMaxW + q], src[size_t(j) * ncol + c], acc);
  }
  dst[size_t(i) * ncol + c] = acc;
}

// Independent transposed projections of one kind in one launch, blockIdx.y picking the job. A job may
// run in place (in == out): each thread owns one column and reads every row of it before writing it.
constexpr int kProjTJobs = 8;
struct ProjTJobs {
  const double2* in[kProjTJobs];
  double2* out[kProjTJobs];
};
// Rows of the sweep loaded this many steps ahead of the dependent chain: at the small sizes this
// kernel runs at, a few waves per CU wait on every row's HBM latency otherwise. The sweeps run in
// blocks of kProjTPre steps, unrolled, so that step d of a block consumes slot d of the ring and then
// refills it, unconditionally (the row index clamped to the sweep's last row): a load's destination
// is then never copied or merged before it is consumed, either of which makes the wave wait for it.
constexpr int kProjTPre = 4;

// (A^{-1} R)^T = R A^{-T} per column, A = L U of the projection `kind`: U^T z = y ascending, L^T x = z
// descending (x in out), then the end rows zeroed for the Dirichlet / Neumann kinds
__global__ void __launch_bounds__(kThreads) k_project_t(DevPlan P, int kind, ProjTJobs J) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const double2* in = J.in[blockIdx.y];
  double2* out = J.out[blockIdx.y];
  const int n2 = P.n2;
  // the factors by columns: row i holds the band entries step i reads (zero outside the matrix, where
  // the ring holds zeros as well, so every term can be formed)
  const auto UT = P.lu_ut + size_t(kind) * n2 * (kMaxBand + 1);
  const auto LT = P.lu_lt + size_t(kind) * n2 * kMaxBand;
  const int nfull = n2 - n2 % kProjTPre;  // steps run in whole blocks; the rest from the ring alone
  double2 ring[kMaxBand];
  double2 pv[kProjTPre];  // slot d: the next row of the sweep whose index is d (mod kProjTPre) from its start
  // U^T z = y: ring[q] = z_{i-1-q}; U_{i-1-q, i} is entry q of row i of UT, 1/U_ii its last
  auto up = [&](int i, double2 b) {
#pragma unroll
    for (int q = 0; q < kMaxBand; ++q) b = fma2(-UT[i * (kMaxBand + 1) + q], ring[q], b);
    const double2 z = cscale(b, UT[i * (kMaxBand + 1) + kMaxBand]);
#pragma unroll
    for (int q = kMaxBand - 1; q > 0; --q) ring[q] = ring[q - 1];
    ring[0] = z;
    out[size_t(i) * ncol + c] = z;
  };
  // L^T x = z: ring[m] = x_{i+1+m}; L_{i+1+m, i} is entry m of row i of LT
  auto down = [&](int i, double2 x) {
#pragma unroll
    for (int m = 0; m < kMaxBand; ++m) x = fma2(-LT[i * kMaxBand + m], ring[m], x);
#pragma unroll
    for (int m = kMaxBand - 1; m > 0; --m) ring[m] = ring[m - 1];
    ring[0] = x;
    out[size_t(i) * ncol + c] = (kind != 0 && (i == 0 || i == n2 - 1)) ? zero2() : x;
  };
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) ring[m] = zero2();
#pragma unroll
  for (int d = 0; d < kProjTPre; ++d) pv[d] = in[size_t(min(d, n2 - 1)) * ncol + c];
  for (int i0 = 0; i0 < nfull; i0 += kProjTPre) {
#pragma unroll
    for (int d = 0; d < kProjTPre; ++d) {
      const int i = i0 + d;
      up(i, pv[d]);
      pv[d] = in[size_t(min(i + kProjTPre, n2 - 1)) * ncol + c];
    }
  }
#pragma unroll
  for (int d = 0; d < kProjTPre; ++d)
    if (nfull + d < n2) up(nfull + d, pv[d]);
#pragma unroll
  for (int m = 0; m < kMaxBand; ++m) ring[m] = zero2();
  // descending over z (written above by this thread): step d of a block is row n2 - 1 - (i0 + d)
#pragma unroll
  for (int d = 0; d < kProjTPre; ++d) pv[d] = out[size_t(max(n2 - 1 - d, 0)) * ncol + c];
  for (int i0 = 0; i0 < nfull; i0 += kProjTPre) {
#pragma unroll
    for (int d = 0; d < kProjTPre; ++d) {
      const int i = n2 - 1 - (i0 + d);
      down(i, pv[d]);
      pv[d] = out[size_t(max(i - kProjTPre, 0)) * ncol + c];
    }
  }
#pragma unroll
  for (int d = 0; d < kProjTPre; ++d)
    if (nfull + d < n2) down(n2 - 1 - (nfull + d), pv[d]);
}

constexpr int kFacMax = 9;  // band of the factor rows (a_lower, a_upper <= 8)
constexpr int kScatPre = 4;  // psi rows read ahead by scatter_Gt
// psi = A(k)^{-T} b in place in scr (n2 + 1 rows of column c), A = U L from the plan's factors of pair
// fac (U unit upper: the multipliers; L: entries left of the diagonal and the inverse diagonal):
// L^T w = b descending, then U^T psi = w ascending
__device__ __forceinline__ void solve_At(const DevPlan& P, const double* fac, int npairs, double2* scr, size_t c,
                                         size_t ncol) {
  const int N = P.n2 + 1;
  // The operands of a step (the value row and the factor entries it needs) are loaded D = kFacPre steps
  // ahead: at two waves per SIMD or fewer the HBM latency is otherwise exposed at every step of the
  // chain. The sweeps run in unrolled blocks of D steps; step d of a block consumes ring slot d and then
  // refills it with unconditional loads at in-range addresses (entries outside a row's band are masked
  // where they are used), so a load keeps its register until its use.
  constexpr int D = kFacPre;
  const int nfull = N - N % D;
  double fr[D][kFacMax + 1];
  double2 pv[D];
  double2 ring[kFacMax];
  // L^T w = b (descending): ring[q] = w_{i+1+q}; L_{i+1+q, i} is left entry q of row i+1+q, at the slot
  // the plan's column table gives (-1: none; slot 0 is read instead and masked at use)
  auto load_lt = [&](double (&e)[kFacMax + 1], int i) __attribute__((always_inline)) {
    const auto sl = P.fac_lt + size_t(max(i, 0)) * (kFacMax + 1);
#pragma unroll
    for (int q = 0; q <= kFacMax; ++q) e[q] = fac[size_t(max(sl[q], 0)) * npairs];
  };
  auto step_lt = [&](int i, double2 b, const double (&e)[kFacMax + 1]) __attribute__((always_inline)) {
    const auto sl = P.fac_lt + size_t(i) * (kFacMax + 1);
#pragma unroll
    for (int q = 0; q < kFacMax; ++q) b = fma2(-(sl[q] >= 0 ? e[q] : 0.0), ring[q], b);
    const double2 w = cscale(b, e[kFacMax]);
#pragma unroll
    for (int q = kFacMax - 1; q > 0; --q) ring[q] = ring[q - 1];
    ring[0] = w;
    scr[size_t(i) * ncol + c] = w;
  };
#pragma unroll
  for (int q = 0; q < kFacMax; ++q) ring[q] = zero2();
#pragma unroll
  for (int d = 0; d < D; ++d) {  // step t = d (mod D) is row i = N - 1 - t
    load_lt(fr[d], N - 1 - d);
    pv[d] = scr[size_t(max(N - 1 - d, 0)) * ncol + c];
  }
  for (int t0 = 0; t0 < nfull; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = N - 1 - (t0 + d);
      step_lt(i, pv[d], fr[d]);
      load_lt(fr[d], i - D);
      pv[d] = scr[size_t(max(i - D, 0)) * ncol + c];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nfull + d < N) step_lt(N - 1 - (nfull + d), pv[d], fr[d]);
  // U^T psi = w (ascending): ring[m] = psi_{i-1-m}; U_{i-1-m, i} is multiplier m of row i-1-m, at the
  // slot of the plan's column table
  auto load_ut = [&](double (&e)[kFacMax + 1], int i) __attribute__((always_inline)) {
    const auto sl = P.fac_ut + size_t(min(i, N - 1)) * kFacMax;
#pragma unroll
    for (int m = 0; m < kFacMax; ++m) e[m] = fac[size_t(max(sl[m], 0)) * npairs];
  };
  auto step_ut = [&](int i, double2 x, const double (&e)[kFacMax + 1]) __attribute__((always_inline)) {
    const auto sl = P.fac_ut + size_t(i) * kFacMax;
#pragma unroll
    for (int m = 0; m < kFacMax; ++m) x = fma2(-(sl[m] >= 0 ? e[m] : 0.0), ring[m], x);
#pragma unroll
    for (int m = kFacMax - 1; m > 0; --m) ring[m] = ring[m - 1];
    ring[0] = x;
    scr[size_t(i) * ncol + c] = x;
  };
#pragma unroll
  for (int q = 0; q < kFacMax; ++q) ring[q] = zero2();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    load_ut(fr[d], d);
    pv[d] = scr[size_t(min(d, N - 1)) * ncol + c];
  }
  for (int i0 = 0; i0 < nfull; i0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = i0 + d;
      step_ut(i, pv[d], fr[d]);
      load_ut(fr[d], i + D);
      pv[d] = scr[size_t(min(i + D, N - 1)) * ncol + c];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nfull + d < N) step_ut(nfull + d, pv[d], fr[d]);
}

// out (n2 rows of column c) = (add ? out : 0) + sum over the interior tau* rows i of G_g[i, :]^T scale psi_i
// (g = 0: G0, 1: G1); the rows each tau* row reaches start at a nondecreasing position, so finished rows
// leave a register window in order
__device__ __forceinline__ void scatter_Gt(const DevPlan& P, int g, const double2* scr, double scale, double2* out,
                                           size_t c, size_t ncol, bool add) {
  const int n2 = P.n2, N = n2 + 1;
  double2 acc[kMaxW];
#pragma unroll
  for (int q = 0; q < kMaxW; ++q) acc[q] = zero2();
  int base = 0;
  // the row that leaves the window next, read one row ahead (from scr, valid and unused, without add)
  const double2* osrc = add ? out : scr;
  double2 onext = osrc[c];
  auto flush = [&]() __attribute__((always_inline)) {
    const size_t e = size_t(base) * ncol + c;
    const double2 o = add ? cadd(onext, acc[0]) : acc[0];
    onext = osrc[size_t(min(base + 1, n2 - 1)) * ncol + c];
    out[e] = o;
#pragma unroll
    for (int q = 0; q < kMaxW - 1; ++q) acc[q] = acc[q + 1];
    acc[kMaxW - 1] = zero2();
    ++base;
  };
  auto step = [&](int i, double2 pr) __attribute__((always_inline)) {
    const int lo = P.gs_lo[g * N + i];
    while (base < lo) flush();
    const double2 psi = cscale(pr, scale);
#pragma unroll
    for (int q = 0; q < kMaxW; ++q)
      if (lo + q < n2) acc[q] = fma2(P.gs_w[(size_t(g) * N + i) * kMaxW + q], psi, acc[q]);
  };
  // psi rows 1 .. n2 - 1 through a ring like solve_At's: step t is row i = 1 + t, slot t mod kScatPre
  constexpr int D = kScatPre;
  const int nsteps = n2 - 1, nfull = nsteps - nsteps % D;
  double2 pf[D];
#pragma unroll
  for (int d = 0; d < D; ++d) pf[d] = scr[size_t(min(1 + d, n2 - 1)) * ncol + c];
  for (int t0 = 0; t0 < nfull; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int i = 1 + t0 + d;
      step(i, pf[d]);
      pf[d] = scr[size_t(min(i + D, n2 - 1)) * ncol + c];
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (nfull + d < nsteps) step(1 + nfull + d, pf[d]);
  while (base < n2) flush();
}

// transpose of the m^d map (phi2, Omega2, <m>1, <m>3) -> (m1, m2, m3) coefficients (eqs. phi_poisson,
// bc_both, md_recon).  Per column: the adjoints of D = D* c and of Omega2 from the m1, m3 adjoints (the
// multipliers i k1 / k^2, i k3 / k^2 conjugated), c_bar = m2_bar + D*^T D_bar, psi = A(k)^{-T} c_bar with
// the plan's factors A = U L (U unit upper: the multipliers, L: entries left of the diagonal and the
// inverse diagonal) as L^T w = c_bar descending and U^T psi = w ascending, then phi2_bar = G0^T psi over
// the interior tau* rows (the Robin rows carry no phi2).  psi goes through scr (n2 + 1 rows).
__global__ void __launch_bounds__(kThreads) k_md_t(DevPlan P, const double2* __restrict__ a1,
                                                  const double2* __restrict__ a2, const double2* __restrict__ a3,
                                                  double2* __restrict__ phi_t, double2* __restrict__ om_t,
                                                  double* __restrict__ m1bar_t, double* __restrict__ m3bar_t,
                                                  double2* __restrict__ scr) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const size_t ncol = size_t(nn) * nl;
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int l = int(c % size_t(nl)), ni = int(c / size_t(nl));
  const double k1 = P.k1[l], k3 = P.k3[ni], ksq = k1 * k1 + k3 * k3;
  if (ksq == 0.0) {  // (0,0): m1 = <m>1, m3 = <m>3, m2 = 0; phi2, Omega2 do not enter
    for (int i = 0; i < n2; ++i) {
      m1bar_t[i] = a1[size_t(i) * ncol].x;
      m3bar_t[i] = a3[size_t(i) * ncol].x;
      phi_t[size_t(i) * ncol] = zero2();
      om_t[size_t(i) * ncol] = zero2();
    }
    return;
  }
  const double iksq = 1.0 / ksq;
  const int half = (nn + 1) / 2, npairs = nl * half;
  const int pp = ni < half ? ni : nn - ni;
  const double* fac = P.fac + size_t(pp) * nl + l;
  // c_bar = m2_bar + D*^T D_bar; Omega2_bar
  double2 dprev = zero2();
  for (int r = 0; r < N; ++r) {
    double2 db = zero2();
    if (r < n2) {
      const double2 m1 = a1[size_t(r) * ncol + c], m3 = a3[size_t(r) * ncol + c];
      db = cscale(times_i(make_double2(-(k1 * m1.x + k3 * m3.x), -(k1 * m1.y + k3 * m3.y))), iksq);
      om_t[size_t(r) * ncol + c] = cscale(times_i(make_double2(k3 * m1.x - k1 * m3.x, k3 * m1.y - k1 * m3.y)), iksq);
    }
    double2 cb = a2[size_t(r) * ncol + c];
    if (r >= 1) cb = fma2(P.dstar[r - 1], dprev, cb);
    if (r < n2) cb = fma2(-P.dstar[r], db, cb);
    scr[size_t(r) * ncol + c] = cb;
    dprev = db;
  }
  solve_At(P, fac, npairs, scr, c, ncol);
  scatter_Gt(P, 0, scr, 1.0, phi_t, c, ncol, false);
}

// transpose of the m^c map rho_t (B coefficients) -> (m1, m2, m3) (eqs. COM_fourier, CF_fourier, mc_recon,
// mc_mean): m_par_bar = (k1 m1_bar + k3 m3_bar) / k; rho_t_bar = D_bar = (-i/k) m_par_bar; c_bar = m2_bar +
// D*^T D_bar; psi = A(k)^{-T} c_bar; rho_t_bar -= G1^T psi over the interior rows.  The (0,0) column solves
// the transposed mean system [D*; top row]^T psi = m2_bar by one ascending recurrence, rho_t_bar = -psi.
__global__ void __launch_bounds__(kThreads) k_mc_t(DevPlan P, const double2* __restrict__ a1,
                                                  const double2* __restrict__ a2, const double2* __restrict__ a3,
                                                  double2* __restrict__ rho_t, double2* __restrict__ scr) {
  const int nl = P.nl, nn = P.nn, n2 = P.n2, N = n2 + 1;
  const size_t ncol = size_t(nn) * nl;
  const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int l = int(c % size_t(nl)), ni = int(c / size_t(nl));
  const double k1 = P.k1[l], k3 = P.k3[ni], ksq = k1 * k1 + k3 * k3;
  if (ksq == 0.0) {
    // psi_0 = -b_0 / d_0; psi_r = (d_{r-1} psi_{r-1} - b_r) / d_r (r < n2); rho_t_bar_r = -psi_r
    double2 prev = zero2();
    for (int r = 0; r < n2; ++r) {
      double2 b = a2[size_t(r) * ncol];
      if (r >= 1) b = make_double2(P.dstar[r - 1] * prev.x - b.x, P.dstar[r - 1] * prev.y - b.y);
      else b = make_double2(-b.x, -b.y);
      prev = cscale(b, 1.0 / P.dstar[r]);
      rho_t[size_t(r) * ncol] = make_double2(-prev.x, -prev.y);
    }
    return;
  }
  const double ik = 1.0 / sqrt(ksq);
  const int half = (nn + 1) / 2, npairs = nl * half;
  const int pp = ni < half ? ni : nn - ni;
  const double* fac = P.fac + size_t(pp) * nl + l;
  double2 dprev = zero2();
  for (int r = 0; r < N; ++r) {
    double2 db = zero2();
    if (r < n2) {
      const double2 m1 = a1[size_t(r) * ncol + c], m3 = a3[size_t(r) * ncol + c];
      const double2 mp = make_double2((k1 * m1.x + k3 * m3.x) * ik, (k1 * m1.y + k3 * m3.y) * ik);
      db = cscale(make_double2(mp.y, -mp.x), ik);  // (-i/k) m_par_bar
      rho_t[size_t(r) * ncol + c] = db;
    }
    double2 cb = a2[size_t(r) * ncol + c];
    if (r >= 1) cb = fma2(P.dstar[r - 1], dprev, cb);
    if (r < n2) cb = fma2(-P.dstar[r], db, cb);
    scr[size_t(r) * ncol + c] = cb;
    dprev = db;
  }
  solve_At(P, fac, npairs, scr, c, ncol);
  scatter_Gt(P, 1, scr, -1.0, rho_t, c, ncol, true);  // rho_t_bar -= G1^T psi
}

// the inverse transform's transpose from the forward one: times M1 M3, and 2 for l > 0 (a real field
// takes c_l and its conjugate partner -l; the l = 0 column enters through its real part)
// (inv = 1: the forward transform's transpose divides instead, before an inverse transform)
__global__ void __launch_bounds__(kThreads) k_scale_modes(DevPlan P, const double2* __restrict__ src,
                                                         double2* __restrict__ v, int inv) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ncol * P.n2) return;
  const int l = int(e % size_t(P.nl));
  const double f = double(P.m1) * double(P.m3) * (l == 0 ? 1.0 : 2.0);
  v[e] = cscale(src[e], inv ? 1.0 / f : f);
}

// ---------------------------------------------------------------------------
// host side

#define HIP_OK(x)                                    \
  do {                                               \
    if ((x) != hipSuccess) return LMVD_EHIP;         \
  } while (0)

struct Workspace {
  size_t bytes = 0;
  size_t off_md1, off_md3, off_c2d, off_mpar, off_c2c, off_rz, off_zta, off_ztb, off_rhot, off_vals[kMaxOut];
  size_t off_u[3], off_T[6], off_rhov, off_yphi, off_yom, off_uscr, off_zbuf, off_obuf, off_aux;
  size_t off_yp, off_yt;  // scratch of the m^c column kernel
  // values at the Greville points
  size_t off_vz0, off_vz1, off_vzl, off_vz3, off_vmd1, off_vmd3, off_vc2d, off_vm1c, off_vm2c, off_vm3c, off_vzt;
  size_t off_szt = 0;  // filtered R_z values, x-spectral and z-physical (elided fixed-point path)
};

}  // namespace lmvd

struct lmvd_prof {
  int cls = -1;                 // kernel class being timed, -1 = off
  std::vector<hipEvent_t> ev;   // start/stop pairs
  int used = 0;                 // pairs recorded
  double bytes = 0.0;           // compulsory bytes of the recorded launches
};

struct lmvd_plan_s {
  lmvd::HostTables H;
  lmvd_prof prof;
  lmvd::DevPlan D{};
  std::vector<void*> allocs;
  lmvd::Workspace ws;
  int pb = 0;       // planes per batch
  int lgz = 1;      // l-lines per z-FFT block
  int bgx = 1;      // z-lines per x-pass block
  int device = 0;
  bool use_reg = true;  // register-FFT kernels for the specialised sizes
  double* fac = nullptr;    // A(k) factors (plan memory), computed and checked at plan creation
  int fac_la = 7, fac_ua = 7;  // instantiated band of the factor kernels
  double fac_growth = 0.0, fac_pivot = 0.0;  // largest growth, smallest pivot ratio of the check
  int64_t fac_bad = 0;      // rows that failed the check
  unsigned* finite_flag = nullptr;  // device words: the non-finite scan (0), the factor check (16..18)
  int zdiv = 1;     // z tile divisor of the register z kernels below 768 points (lmvd_autotune)
};

namespace lmvd {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static void layout_workspace(lmvd_plan_s* p) {
  const HostTables& H = p->H;
  const size_t ncol = size_t(H.nn) * H.nl;
  const size_t sB = ncol * H.n2 * 16, sS = ncol * (H.n2 + 1) * 16;
  const int UPA = 8;  // widest instantiation of k_solveA (band 8, 8)
  size_t o = 0;
  Workspace& w = p->ws;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  w.off_md1 = take(sB);
  w.off_md3 = take(sB);
  w.off_c2d = take(sS);
  w.off_mpar = take(sB);
  w.off_c2c = take(sS);
  w.off_rz = take(sB);
  w.off_zta = take(sB);
  w.off_ztb = take(sB);
  w.off_rhot = take(sB);
  for (int g = 0; g < kMaxOut; ++g) w.off_vals[g] = take(sB);
  for (int i = 0; i < 3; ++i) w.off_u[i] = take(sB);
  for (int i = 0; i < 6; ++i) w.off_T[i] = take(sB);
  w.off_rhov = take(sB);
  w.off_yphi = take(sB);
  w.off_yom = take(sB);
  const size_t npairs = size_t(H.nl) * ((H.nn + 1) / 2);
  w.off_uscr = take(size_t(H.n2 + 1) * (UPA + 1) * npairs * 8);
  const size_t plane = size_t(H.cfg.m3) * H.nl * 16;
  w.off_zbuf = take(size_t(kMaxIn) * p->pb * plane);
  w.off_obuf = take(size_t(kMaxOut) * p->pb * plane);
  w.off_yp = take(sB);
  w.off_yt = take(sS);
  w.off_aux = take(size_t(kNumAux) * H.n2 * H.cfg.m3 * H.cfg.m1 * 8);
  w.off_vz0 = take(sB);
  w.off_vz1 = take(sB);
  w.off_vzl = take(sB);
  w.off_vz3 = take(sB);
  w.off_vmd1 = take(sB);
  w.off_vmd3 = take(sB);
  w.off_vc2d = take(sB);
  w.off_vm1c = take(sB);
  w.off_vm2c = take(sB);
  w.off_vm3c = take(sB);
  w.off_vzt = take(sB);
  if (p->pb == H.n2) w.off_szt = take(plane * H.n2);
  w.bytes = o;
}

template <typename T>
static lmvd_status upload(lmvd_plan_s* p, const std::vector<T>& v, const T** dst) {
  void* d = nullptr;
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  if (hipMalloc(&d, bytes) != hipSuccess) return LMVD_ENOMEM;
  p->allocs.push_back(d);
  if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return LMVD_EHIP;
  *dst = static_cast<const T*>(d);
  return LMVD_OK;
}

static void cat_rows(const RowTable* t, int count, std::vector<int>& lo, std::vector<double>& w) {
  for (int k = 0; k < count; ++k) {
    lo.insert(lo.end(), t[k].lo.begin(), t[k].lo.end());
    w.insert(w.end(), t[k].w.begin(), t[k].w.end());
  }
}

static void fill_fft(const FftPlan& f, FftDev& d) {
  d.n = f.n;
  d.nstages = f.nstages;
  for (int s = 0; s < kMaxStagesDev; ++s) {
    d.radix[s] = s < f.nstages ? f.radix[s] : 0;
    d.ns[s] = s < f.nstages ? f.ns[s] : 0;
  }
}

// choose launch shapes
static void choose_shapes(lmvd_plan_s* p) {
  const HostTables& H = p->H;
  const int M3 = H.cfg.m3;
  // l-lines per z-FFT block: at most 64 KiB of LDS and kZMaxE elements per thread
  int lg = std::max(1, std::min(4096, kZMaxE * kThreads) / M3);  // kZMaxE * kThreads = 3072
  int pw = 1;
  while (pw * 2 <= lg) pw *= 2;
  lg = std::min(pw, H.nl);
  p->lgz = lg;
  int bg = std::max(1, (kXSlots * kThreads) / H.hx);
  bg = std::min(bg, M3);
  p->bgx = bg;
}

static lmvd_status factor_and_check(lmvd_plan_s* p, double growth_max);

// Workspace of lmvd_substep_noalloc: one array in device memory per GPU, held until the process ends.
// In host code `scratch` is only a host-side stand-in for the symbol; its device address on each GPU
// comes from hipGetSymbolAddress (resolve_scratch, at plan creation with the plan's device current) and
// only that address is handed to kernels.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
static void* scratch_ptr[kMaxDevices] = {};
static std::mutex scratch_mu;

static lmvd_status resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return LMVD_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return LMVD_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LMVD_EHIP;
  scratch_ptr[device] = ptr;
  return LMVD_OK;
}

static void* device_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_ptr[device];
}

static lmvd_status create_plan(const lmvd_config* cfg, lmvd_plan* out, std::string& msg) {
  if (!cfg || !out) return LMVD_EINVAL;
  lmvd_plan_s* p = new (std::nothrow) lmvd_plan_s();
  if (!p) return LMVD_ENOMEM;
  lmvd_status st = build_host_tables(*cfg, p->H, msg);
  if (st != LMVD_OK) {
    delete p;
    return st;
  }
  HostTables& H = p->H;
  // k_xpass stages one x-line of m1/2 complex values in kXSlots * kThreads slots
  if (H.nl > H.hx || H.nn > cfg->m3 || H.hx > kXSlots * kThreads) {
    delete p;
    return LMVD_EUNSUPPORTED;
  }
  if (H.a_lower > 8 || H.a_upper > 8) {
    delete p;
    return LMVD_EUNSUPPORTED;
  }
  // the plane-mean kernel keeps both components' rows in 64 KB of LDS
  if (size_t(2) * H.n2 * sizeof(double) > 65536) {
    msg = "n2 above 4096 is not supported";
    delete p;
    return LMVD_EUNSUPPORTED;
  }
  if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
  st = resolve_scratch(p->device);
  if (st != LMVD_OK) {
    msg = "device address of the allocation-free workspace";
    delete p;
    return st;
  }
  p->pb = (cfg->plane_batch > 0) ? std::min(cfg->plane_batch, H.n2) : H.n2;
  choose_shapes(p);
  DevPlan& D = p->D;
  D.n2 = H.n2;
  D.p = H.p;
  D.nl = H.nl;
  D.nn = H.nn;
  D.n3 = cfg->n3;
  D.m1 = cfg->m1;
  D.m3 = cfg->m3;
  D.hx = H.hx;
  D.dt = cfg->dt;
  D.mu = cfg->mu;
  D.rhoD = cfg->rhoD;
  D.g = cfg->g;
  D.rho_l = cfg->rho_l;
  D.rho_h = cfg->rho_h;
  D.inv_rlrh = 1.0 / (cfg->rho_l * cfg->rho_h);
  D.drho = cfg->rho_h - cfg->rho_l;
  for (int k = 0; k < 3; ++k) {
    D.mu_z[k] = cfg->mu_z[k];
    D.rq_z[k] = cfg->rhoD_z[k];
  }
  D.rq_form = cfg->rhoD_form;
  std::vector<int> lo;
  std::vector<double> w;
  RowTable ev[kNumEv] = {H.E[0], H.E[1], H.E[2], H.F0};
  cat_rows(ev, kNumEv, lo, w);
#define UP_OR_FAIL(vec, dst)                \
  do {                                      \
    st = upload(p, vec, dst);               \
    if (st != LMVD_OK) {                    \
      lmvd_plan_destroy(p);                 \
      return st;                            \
    }                                       \
  } while (0)
  // tables read through the constant address space
#define UP_TABLE(vec, member)                                      \
  do {                                                             \
    const std::remove_reference_t<decltype(vec[0])>* tmp_ = nullptr; \
    UP_OR_FAIL(vec, &tmp_);                                        \
    member = (decltype(member))(tmp_);                             \
  } while (0)
  UP_TABLE(lo, D.ev_lo);
  UP_TABLE(w, D.ev_w);
  lo.clear();
  w.clear();
  cat_rows(H.G, 2, lo, w);
  UP_TABLE(lo, D.gs_lo);
  UP_TABLE(w, D.gs_w);
  lo.clear();
  w.clear();
  cat_rows(H.Es, 3, lo, w);
  UP_TABLE(lo, D.es_lo);
  UP_TABLE(w, D.es_w);
  UP_TABLE(H.dstar, D.dstar);
  std::vector<double> L, U, Ui;
  for (int k = 0; k < 3; ++k) {
    L.insert(L.end(), H.proj[k].lmul.begin(), H.proj[k].lmul.end());
    U.insert(U.end(), H.proj[k].u.begin(), H.proj[k].u.end());
    Ui.insert(Ui.end(), H.proj[k].uinv.begin(), H.proj[k].uinv.end());
  }
  UP_TABLE(L, D.lu_l);
  UP_TABLE(U, D.lu_u);
  UP_TABLE(Ui, D.lu_uinv);
  // the same factors by columns, for the transposed sweeps: what a step of U^T z = y or L^T x = z reads
  // is one contiguous row (one scalar-load batch per step instead of one load per band row)
  {
    const int n2 = H.n2;
    std::vector<double> UT(size_t(3) * n2 * (kMaxBand + 1), 0.0), LT(size_t(3) * n2 * kMaxBand, 0.0);
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < n2; ++i) {
        double* ut = &UT[(size_t(k) * n2 + i) * (kMaxBand + 1)];
        double* lt = &LT[(size_t(k) * n2 + i) * kMaxBand];
        for (int q = 0; q < kMaxBand; ++q) {
          if (i - 1 - q >= 0) ut[q] = U[(size_t(k) * n2 + i - 1 - q) * (kMaxBand + 1) + q + 1];
          if (i + 1 + q < n2) lt[q] = L[(size_t(k) * n2 + i + 1 + q) * kMaxBand + q];
        }
        ut[kMaxBand] = Ui[size_t(k) * n2 + i];
      }
    UP_TABLE(UT, D.lu_ut);
    UP_TABLE(LT, D.lu_lt);
  }
  UP_OR_FAIL(H.k1, &D.k1);
  UP_OR_FAIL(H.k3, &D.k3);
  UP_TABLE(H.emit_first, D.emit_first);
  UP_TABLE(H.emit_cnt, D.emit_cnt);
  UP_TABLE(H.g1e_cnt, D.g1e_cnt);
  UP_TABLE(H.asc_first, D.asc_first);
  UP_TABLE(H.asc_cnt, D.asc_cnt);
  UP_TABLE(H.asc_w, D.asc_w);
  UP_TABLE(H.fac_nm, D.fac_nm);
  UP_TABLE(H.fac_ns, D.fac_ns);
  UP_TABLE(H.fac_off, D.fac_off);
  {
    const int N = H.n2 + 1;
    std::vector<int32_t> lt(size_t(N) * (kFacMax + 1), -1), ut(size_t(N) * kFacMax, -1);
    for (int i = 0; i < N; ++i) {
      for (int q = 0; q < kFacMax; ++q) {
        const int r = i + 1 + q;
        if (r < N && q < H.fac_ns[r]) lt[size_t(i) * (kFacMax + 1) + q] = H.fac_off[r] + H.fac_nm[r] + q;
        const int u = i - 1 - q;
        if (u >= 0 && q < H.fac_nm[u]) ut[size_t(i) * kFacMax + q] = H.fac_off[u] + q;
      }
      lt[size_t(i) * (kFacMax + 1) + kFacMax] = H.fac_off[i] + H.fac_nm[i] + H.fac_ns[i];
    }
    UP_TABLE(lt, D.fac_lt);
    UP_TABLE(ut, D.fac_ut);
  }
  UP_TABLE(H.wall_w, D.wall_w);
  D.wall_k0 = H.wall_k0;
  D.wall_k1 = H.wall_k1;
  {
    p->fac_la = p->fac_ua = (H.a_lower <= 7 && H.a_upper <= 7) ? 7 : 8;
    const size_t npairs = size_t(H.nl) * ((H.nn + 1) / 2);
    const size_t bytes = size_t(H.fac_slots) * npairs * sizeof(double);
    void* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) {
      lmvd_plan_destroy(p);
      return LMVD_ENOMEM;
    }
    p->allocs.push_back(d);
    p->fac = static_cast<double*>(d);
    D.fac = p->fac;
  }
  {
    void* d = nullptr;
    if (hipMalloc(&d, 256) != hipSuccess) {
      lmvd_plan_destroy(p);
      return LMVD_ENOMEM;
    }
    p->allocs.push_back(d);
    p->finite_flag = static_cast<unsigned*>(d);
  }
  const double* tw = nullptr;
  UP_OR_FAIL(H.fz.tw, &tw);
  fill_fft(H.fz, D.fz);
  D.fz.tw = reinterpret_cast<const double2*>(tw);
  UP_OR_FAIL(H.fx.tw, &tw);
  fill_fft(H.fx, D.fx);
  D.fx.tw = reinterpret_cast<const double2*>(tw);
  UP_OR_FAIL(H.xtw, &tw);
  D.xtw = reinterpret_cast<const double2*>(tw);
#undef UP_TABLE
#undef UP_OR_FAIL
  st = factor_and_check(p, kGrowthMax);
  if (st != LMVD_OK) {
    if (st == LMVD_ENUMERIC) msg = "A(k) fails the pivot check without pivoting";
    lmvd_plan_destroy(p);
    return st;
  }
  layout_workspace(p);
  *out = p;
  return LMVD_OK;
}

// ---------------------------------------------------------------------------
// launchers

struct Recorder;
struct Ctx {
  lmvd_plan_s* p;
  char* ws;
  hipStream_t s;
  Recorder* rec = nullptr;  // set: launches are recorded for a grouped graph, not issued
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

static size_t ncols(const lmvd_plan_s* p) { return size_t(p->H.nn) * p->H.nl; }

// ---------------------------------------------------------------------------
// Launch routing.  With no recorder a launch happens at once on the context's
// stream.  With a recorder (the grouped mode of lmvd_graph_create) the
// substep's launches are collected per instance: column jobs as argument
// records, to be issued later as one grouped launch over all instances, and
// everything else (plane phases, per-instance kernels) as functions to run on
// that instance's stream.

struct JobOps {  // type-erased job: record size, packing, grouped launch
  size_t rec_size;
  void (*pack)(void* dst, const void* args, int inst, unsigned b0, dim3 grid);
  void (*launch)(const DevPlan* plans, const void* recs, int nrec, unsigned blocks, size_t lds, hipStream_t s);
};

template <class Job>
struct JobOpsOf {
  using A = typename Job::Args;
  static void pack(void* dst, const void* args, int inst, unsigned b0, dim3 g) {
    GRec<A> r;
    std::memcpy(&r.a, args, sizeof(A));
    r.inst = inst;
    r.b0 = b0;
    r.nbx = g.x;
    r.nby = g.y;
    std::memcpy(dst, &r, sizeof(r));
  }
  static void launch(const DevPlan* plans, const void* recs, int nrec, unsigned blocks, size_t lds, hipStream_t s) {
    if constexpr (Job::kMinBlocks > 0)
      hipLaunchKernelGGL(k_group_mb<Job>, dim3(blocks), dim3(Job::kBlock), lds, s, plans,
                         static_cast<const GRec<A>*>(recs), nrec);
    else
      hipLaunchKernelGGL(k_group<Job>, dim3(blocks), dim3(Job::kBlock), lds, s, plans,
                         static_cast<const GRec<A>*>(recs), nrec);
  }
  static const JobOps ops;
};
template <class Job>
const JobOps JobOpsOf<Job>::ops = {sizeof(GRec<typename Job::Args>), &JobOpsOf<Job>::pack, &JobOpsOf<Job>::launch};

struct RecOp {
  const JobOps* job = nullptr;  // column job, or nullptr for a function
  std::vector<unsigned char> args;
  dim3 grid;
  size_t lds = 0;
  std::function<lmvd_status(hipStream_t)> fn;
};
struct Recorder {
  std::vector<RecOp> ops;
};

// a column job: launched now, or recorded for a grouped launch
template <class Job>
static void col(const Ctx& c, dim3 grid, size_t lds, const typename Job::Args& A) {
  if (!c.rec) {
    Job::launch(grid, lds, c.s, c.p->D, A);
    return;
  }
  RecOp op;
  op.job = &JobOpsOf<Job>::ops;
  op.args.resize(sizeof(A));
  std::memcpy(op.args.data(), &A, sizeof(A));
  op.grid = grid;
  op.lds = lds;
  c.rec->ops.push_back(std::move(op));
}

// anything else: run now, or recorded as a function of the instance's stream
template <class F>
static lmvd_status per_instance(const Ctx& c, F&& f) {
  if (!c.rec) return f(c);
  const Ctx base{c.p, c.ws, nullptr, nullptr};
  RecOp op;
  op.fn = [base, f](hipStream_t s) {
    Ctx cc = base;
    cc.s = s;
    return f(cc);
  };
  c.rec->ops.push_back(std::move(op));
  return LMVD_OK;
}


// kernel classes of the timing hook
// Each class is one kernel (one symbol on the rt512-like sizes); the bytes a
// launch reports are its compulsory traffic: inputs read once, outputs written
// once, the factor tables, and the stored intermediate of a two-sweep banded
// solve (written by the first sweep, read by the second).  Re-reads through
// the caches are not counted.
enum KClass {
  KC_ZINV = 0,       // inverse z transforms (all phases)
  KC_XPASS_RZ = 1,   // x-pass of R_z (also writes the physical aux fields)
  KC_XPASS_L = 2,    // x-pass of L z_t
  KC_XPASS_RHOT = 3, // x-pass of rho_t
  KC_XPASS_VEL = 4,  // x-pass of u, rho, C_ij
  KC_ZFWD = 5,       // forward z transforms (all phases)
  KC_MC = 6,         // fused m^c column kernel
  KC_MD = 7,         // m^d solve with the z values and the guess in the same launch
  KC_PROJ = 8,       // projection with plain store (u_hat, R_z)
  KC_PROJ_ZT = 9,    // projection + R_z add (+ z update) of the fixed-point iterate
  KC_VALUES = 10,    // values at tau of fixed fields (m^d, z, guess)
  KC_FLUX = 11,      // T_ij projection and RHS emission (both groups)
  KC_RHS = 12,       // RHS projection, RK2 update, plane means
  KC_XPASS_IO = 13,  // x-pass of the transform entry points
  KC_ZFILT = 14,     // z filter and wall planes of the non-final fixed-point iterates
  KC_COUNT = 15
};

// Bracket one launch of class `cls` with events when that class is timed.
struct ProfScope {
  lmvd_plan_s* p;
  hipStream_t s;
  bool on;
  ProfScope(lmvd_plan_s* p_, int cls, hipStream_t s_, double bytes) : p(p_), s(s_) {
    lmvd_prof& f = p->prof;
    on = (f.cls == cls) && (2 * f.used + 1 < int(f.ev.size()));
    if (on) {
      (void)hipEventRecord(f.ev[2 * f.used], s);
      f.bytes += bytes;
    }
  }
  ~ProfScope() {
    if (on) {
      (void)hipEventRecord(p->prof.ev[2 * p->prof.used + 1], s);
      ++p->prof.used;
    }
  }
};

static EvalIn ev(const void* a, int kind, int ma = MU_ONE, const void* b = nullptr, int mb = MU_ONE) {
  EvalIn e;
  e.a = static_cast<const double2*>(a);
  e.b = static_cast<const double2*>(b);
  e.kind = kind;
  e.ma = ma;
  e.mb = mb;
  e.slot = -1;
  return e;
}

// z tile code (D = 1, 2, 4 with plan V = 0, 1, 2: codes D + 8 V; anything else is 1) as a compile-time
// constant
template <typename F>
static void ztile_dispatch(int code, F&& f) {
  switch (code) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 17: f(std::integral_constant<int, 17>{}); break;
    case 18: f(std::integral_constant<int, 18>{}); break;
    case 20: f(std::integral_constant<int, 20>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}
static bool ztile_valid(int code) {
  const int d = code % 8, v = code / 8;
  return (d == 1 || d == 2 || d == 4) && v >= 0 && v <= 2;
}

// register-FFT launches for the specialised sizes
template <int N>
static void launch_zinv_t(const Ctx& c, const EvalArgs& A, double2* zbuf, int j0, int nb, int nin) {
  lmvd_plan_s* p = c.p;
  const bool exact = p->H.nn == 2 * N / 3 - 1;
  if constexpr (N == 768) {
    using ZP = ZPlanW<N>;
    const dim3 g(nin, (p->H.nl + ZP::LG - 1) / ZP::LG, nb);
    const size_t lds = size_t(ZP::LG) * ZP::STRIDE * sizeof(double) +
                       size_t(rf::StageTw<ZP::R0, ZP::R1, ZP::R2, ZP::R3>::SIZE) * sizeof(double2);
    if (exact) col<JobZinvW<N, true>>(c, g, lds, {A, zbuf, j0, p->pb});
    else col<JobZinvW<N, false>>(c, g, lds, {A, zbuf, j0, p->pb});
    return;
  }
  auto go = [&](auto dv) {
    constexpr int D = decltype(dv)::value;
    using ZS = ZShape<N, D>;
    const dim3 g((p->H.nl + ZS::LG - 1) / ZS::LG, nb, nin);
    const size_t lds = size_t(ZS::LG) * ZS::STRIDE * sizeof(double);
    if (exact) col<JobZinvR<N, true, D>>(c, g, lds, {A, zbuf, j0, p->pb});
    else col<JobZinvR<N, false, D>>(c, g, lds, {A, zbuf, j0, p->pb});
  };
  ztile_dispatch(p->zdiv, go);
}
template <int N>
static void launch_zfwd_t(const Ctx& c, const double2* obuf, const OutPtrs& V, int j0, int nb, int nout) {
  lmvd_plan_s* p = c.p;
  if constexpr (N == 768) {
    using ZP = ZPlanW<N>;
    const dim3 g(nout, (p->H.nl + ZP::LG - 1) / ZP::LG, nb);
    const size_t lds = size_t(ZP::LG) * ZP::STRIDE * sizeof(double) +
                       size_t(rf::StageTw<ZP::R0, ZP::R1, ZP::R2, ZP::R3>::SIZE) * sizeof(double2);
    col<JobZfwdW<N>>(c, g, lds, {obuf, V, j0, p->pb});
    return;
  }
  auto go = [&](auto dv) {
    constexpr int D = decltype(dv)::value;
    using ZS = ZShape<N, D>;
    const dim3 g((p->H.nl + ZS::LG - 1) / ZS::LG, nb, nout);
    const size_t lds = size_t(ZS::LG) * ZS::STRIDE * sizeof(double);
    col<JobZfwdR<N, D>>(c, g, lds, {obuf, V, j0, p->pb});
  };
  ztile_dispatch(p->zdiv, go);
}
template <int PH, int N>
static void launch_xpass_t(const Ctx& c, const double2* zbuf, double2* obuf, double* phys_out,
                           const double* phys_in, int j0, int nb, double* aux) {
  lmvd_plan_s* p = c.p;
  using LP = XPlan<N>;
  const dim3 g((p->H.cfg.m3 + LP::BG - 1) / LP::BG, nb);
  const size_t lds = size_t(LP::BG) * LP::STRIDE * sizeof(double) +
                     size_t(rf::StageTw<LP::R0, LP::R1, LP::R2, LP::R3>::SIZE) * sizeof(double2);
  if constexpr (PH == PH_L || PH == PH_RHOT) {
    const dim3 g2((p->H.cfg.m3 + 2 * LP::BG - 1) / (2 * LP::BG), nb);
    col<JobXline<PH, N>>(c, g2, lds, {zbuf, obuf, p->pb, j0, aux});
  } else if constexpr (PH == PH_VEL) {
    col<JobXpair<PH, N, 2>>(c, g, lds, {zbuf, obuf, p->pb, phys_out, phys_in, j0, aux});
  } else {
    col<JobXpair<PH, N, 0>>(c, g, lds, {zbuf, obuf, p->pb, phys_out, phys_in, j0, aux});
  }
}
static bool zreg_size(int n) {
  return n == 768 || n == 192 || n == 144 || n == 96 || n == 72 || n == 48;
}
// full-length x plans; the retained x-modes must be exactly m1/3
static bool xreg_size(int m1, int nl) {
  return (m1 == 768 || m1 == 192 || m1 == 144 || m1 == 96 || m1 == 72 || m1 == 48) && 3 * nl == m1;
}
#define LMVD_ZSWITCH(n, CALL) \
  switch (n) {                \
    case 768: CALL(768); break; \
    case 192: CALL(192); break; \
    case 144: CALL(144); break; \
    case 96: CALL(96); break;   \
    case 72: CALL(72); break;   \
    case 48: CALL(48); break;   \
    default: break;             \
  }
#define LMVD_XSWITCH(n, CALL) \
  switch (n) {                \
    case 768: CALL(768); break; \
    case 192: CALL(192); break; \
    case 144: CALL(144); break; \
    case 96: CALL(96); break;   \
    case 72: CALL(72); break;   \
    case 48: CALL(48); break;   \
    default: break;             \
  }

// zinv = false: the inputs are already in zbuf (x-spectral, z-physical);
// zfwd = false: the outputs stay in obuf.
template <int PH>
static lmvd_status plane_phase(const Ctx& c, const std::vector<EvalIn>& ins, const std::vector<double2*>& outs,
                               double* phys_out = nullptr, const double* phys_in = nullptr, bool zinv = true,
                               bool zfwd = true) {
  lmvd_plan_s* p = c.p;
  const HostTables& H = p->H;
  const int M3 = H.cfg.m3, nl = H.nl;
  EvalArgs A{};
  for (size_t i = 0; i < ins.size(); ++i) {
    A.in[i] = ins[i];
    if (A.in[i].slot < 0) A.in[i].slot = int(i);
  }
  OutPtrs V{};
  for (size_t g = 0; g < outs.size(); ++g) V.v[g] = outs[g];
  double2* zbuf = c.at<double2>(p->ws.off_zbuf);
  double2* obuf = c.at<double2>(p->ws.off_obuf);
  double* aux = c.at<double>(p->ws.off_aux);
  // physical aux fields each phase writes (R_z) or reads (L, rho_t)
  const double naux = (PH == PH_RZ || PH == PH_RZV) ? 4.0 : (PH == PH_L) ? 3.0 : (PH == PH_RHOT) ? 1.0 : 0.0;
  const int lg = p->lgz, bg = p->bgx;
  const size_t lds_z = size_t(lg) * M3 * sizeof(double2);
  const size_t lds_x = size_t(bg) * H.hx * sizeof(double2);
  for (int j0 = 0; j0 < H.n2; j0 += p->pb) {
    const int nb = std::min(p->pb, H.n2 - j0);
    const double zplane = double(M3) * nl * 16.0, splane = double(ncols(p)) * 16.0;
    const double nin = double(ins.size()), nout = double(outs.size());
    bool inputs_plain = true;  // the register z kernels take values with multiplier 1, i k1 or i k3 only
    for (const EvalIn& e : ins)
      if (e.kind != EV_IDENT || (e.ma != MU_ONE && e.ma != MU_IK1 && e.ma != MU_IK3) || (e.b && e.mb != MU_ONE))
        inputs_plain = false;
    const bool zr = p->use_reg && zreg_size(M3) && inputs_plain, xr = p->use_reg && xreg_size(H.cfg.m1, nl);
    if (!ins.empty() && zinv) {
      double terms = 0;
      for (const EvalIn& e : ins) terms += e.b ? 2 : 1;
        ProfScope ps(p, KC_ZINV, c.s, nb * (terms * splane + nin * zplane));
      if (zr) {
#define CALLZ(N) launch_zinv_t<N>(c, A, zbuf, j0, nb, int(ins.size()))
        LMVD_ZSWITCH(M3, CALLZ)
#undef CALLZ
      } else {
        dim3 g1((nl + lg - 1) / lg, nb, int(ins.size()));
        (void)per_instance(c, [=](const Ctx& cc) {
          hipLaunchKernelGGL(k_eval_zinv, g1, dim3(kThreads), lds_z, cc.s, cc.p->D, A, zbuf, j0, cc.p->pb, lg);
          return LMVD_OK;
        });
      }
    }
    {
      constexpr int xcls = (PH == PH_RZ || PH == PH_RZV) ? KC_XPASS_RZ : (PH == PH_L) ? KC_XPASS_L
                           : (PH == PH_RHOT) ? KC_XPASS_RHOT : (PH == PH_VEL || PH == PH_TAU) ? KC_XPASS_VEL
                           : KC_XPASS_IO;
      ProfScope ps(p, xcls, c.s, nb * ((nin + nout) * zplane + naux * double(M3) * H.cfg.m1 * 8.0));
      if (xr) {
#define CALLX(N) launch_xpass_t<PH, N>(c, zbuf, obuf, phys_out, phys_in, j0, nb, aux)
        LMVD_XSWITCH(H.cfg.m1, CALLX)
#undef CALLX
      } else {
        dim3 g2((M3 + bg - 1) / bg, nb);
        (void)per_instance(c, [=](const Ctx& cc) {
          hipLaunchKernelGGL(k_xpass<PH>, g2, dim3(kThreads), lds_x, cc.s, cc.p->D, zbuf, obuf, cc.p->pb, bg,
                             phys_out, phys_in, j0, aux);
          return LMVD_OK;
        });
      }
    }
    if (!outs.empty() && zfwd) {
      ProfScope ps(p, KC_ZFWD, c.s, nb * nout * (zplane + splane));
      if (p->use_reg && zreg_size(M3)) {
#define CALLF(N) launch_zfwd_t<N>(c, obuf, V, j0, nb, int(outs.size()))
        LMVD_ZSWITCH(M3, CALLF)
#undef CALLF
      } else {
        dim3 g3((nl + lg - 1) / lg, nb, int(outs.size()));
        (void)per_instance(c, [=](const Ctx& cc) {
          hipLaunchKernelGGL(k_zfwd, g3, dim3(kThreads), lds_z, cc.s, cc.p->D, obuf, V, j0, cc.p->pb, lg);
          return LMVD_OK;
        });
      }
    }
  }
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

static void proj(const Ctx& c, int kind, const double2* in, double2* out, double2* v0 = nullptr,
                 double2* v1 = nullptr) {
  const int n = int(ncols(c.p));
  // values in, L-sweep intermediate out and back, coefficients out, optional emitted values
  ProfScope ps(c.p, KC_PROJ, c.s, (4.0 + (v0 ? 1.0 : 0.0) + (v1 ? 1.0 : 0.0)) * 16.0 * n * c.p->H.n2);
  col<JobProj<EPI_STORE>>(c, dim3((n + kThreads - 1) / kThreads), 0,
                          {kind, in, out, nullptr, nullptr, nullptr, nullptr, v0, v1, 0, n});
}

template <int MODE>
static void solveA(const Ctx& c, const double2* in1, const double2* in2, const double* m1bar, const double* m3bar,
                   double2* c2, double2* o1, double2* o3) {
  const HostTables& H = c.p->H;
  const int npairs = H.nl * ((H.nn + 1) / 2);
  dim3 grid((npairs + kThreads - 1) / kThreads);
  double* uscr = c.at<double>(c.p->ws.off_uscr);
  const double sB = 16.0 * ncols(c.p) * H.n2, sS = 16.0 * ncols(c.p) * (H.n2 + 1);
  // MODE 0: phi2, Omega2 in, m1, m3 out, c (B*) forward store + read back + final store, U rows stored and read
  const double uscr_bytes = 2.0 * 8.0 * (H.a_upper + 1) * (H.n2 + 1) * double(npairs);
  ProfScope ps(c.p, MODE == 0 ? KC_MD : KC_MC, c.s, (MODE == 0 ? 4.0 * sB : 2.0 * sB) + 3.0 * sS + uscr_bytes);
  // the U scratch stride is (a_upper + 1); kernels are instantiated for the band of the plan
  if (H.a_lower <= 7 && H.a_upper <= 7)
    hipLaunchKernelGGL((k_solveA<MODE, 7, 7>), grid, dim3(kThreads), 0, c.s, c.p->D, in1, in2, m1bar, m3bar, c2, o1,
                       o3, uscr);
  else
    hipLaunchKernelGGL((k_solveA<MODE, 8, 8>), grid, dim3(kThreads), 0, c.s, c.p->D, in1, in2, m1bar, m3bar, c2, o1,
                       o3, uscr);
}

// The plan's A(k) factors for every (l, |n|) pair, with the check of every pivot (k_factor_ul), run on
// the null stream and waited for.  LMVD_ENUMERIC when a row fails the check.
static lmvd_status factor_and_check(lmvd_plan_s* p, double growth_max) {
  const int npairs = p->H.nl * ((p->H.nn + 1) / 2);
  const dim3 g((npairs + kThreads - 1) / kThreads);
  unsigned* stats = p->finite_flag + 16;
  const unsigned init[4] = {0u, 0u, 0x7f800000u, 0u};  // count, max growth (0), min ratio (+inf)
  HIP_OK(hipMemcpy(stats, init, sizeof(init), hipMemcpyHostToDevice));
  if (p->fac_la == 7)
    hipLaunchKernelGGL((k_factor_ul<7, 7>), g, dim3(kThreads), 0, nullptr, p->D, p->fac, growth_max, stats);
  else
    hipLaunchKernelGGL((k_factor_ul<8, 8>), g, dim3(kThreads), 0, nullptr, p->D, p->fac, growth_max, stats);
  HIP_OK(hipGetLastError());
  unsigned h[4];
  HIP_OK(hipMemcpy(h, stats, sizeof(h), hipMemcpyDeviceToHost));
  float gf, rf;
  std::memcpy(&gf, &h[1], 4);
  std::memcpy(&rf, &h[2], 4);
  p->fac_bad = h[0];
  p->fac_growth = gf;
  p->fac_pivot = rf;
  return h[0] ? LMVD_ENUMERIC : LMVD_OK;
}

// out = filter(in) + add on all planes, then the wall planes of out (see k_zfilt_w, k_wall)
static void zfilter(const Ctx& c, const double2* in, const double2* add, double2* out) {
  lmvd_plan_s* p = c.p;
  const HostTables& H = p->H;
  const int M3 = H.cfg.m3, n2 = H.n2;
  const double zf = double(M3) * H.nl * 16.0;
  ProfScope ps(p, KC_ZFILT, c.s, n2 * zf * (add ? 3.0 : 2.0) + zf * (H.wall_k0 + H.wall_k1 + 2));
  if (M3 == 768) {
    using ZP = ZPlanW<768>;
    const size_t lds = size_t(ZP::LG) * ZP::STRIDE * sizeof(double) +
                       size_t(rf::StageTw<ZP::R0, ZP::R1, ZP::R2, ZP::R3>::SIZE) * sizeof(double2);
    col<JobZfiltW<768>>(c, dim3((H.nl + ZP::LG - 1) / ZP::LG, n2), lds, {in, add, out});
  } else {
#define LMVD_ZF(N)                                                                                      \
  ztile_dispatch(p->zdiv, [&](auto dv) {                                                              \
    constexpr int D = decltype(dv)::value;                                                            \
    using ZS = ZShape<N, D>;                                                                          \
    col<JobZfiltR<N, D>>(c, dim3((H.nl + ZS::LG - 1) / ZS::LG, n2), size_t(ZS::LG) * ZS::STRIDE * sizeof(double), \
                         {in, add, out});                                                             \
  })
    switch (M3) {
      case 192: LMVD_ZF(192); break;
      case 144: LMVD_ZF(144); break;
      case 96: LMVD_ZF(96); break;
      case 72: LMVD_ZF(72); break;
      case 48: LMVD_ZF(48); break;
      default: break;
    }
#undef LMVD_ZF
  }
  const size_t ps_ = size_t(M3) * H.nl;
  col<JobWall>(c, dim3(unsigned((ps_ + kThreads - 1) / kThreads)), 0, {out});
}

// transport laws that depend on z
static bool var_mu(const lmvd_config& c) { return c.mu_z[0] != 0.0 || c.mu_z[1] != 0.0 || c.mu_z[2] != 0.0; }
static bool var_rhod(const lmvd_config& c) {
  return c.rhoD_form != 0 || c.rhoD_z[0] != 0.0 || c.rhoD_z[1] != 0.0 || c.rhoD_z[2] != 0.0;
}

// Steps 4 and 5 of the substep (Algorithm time_advanceDNS), shared by lmvd_substep and lmvd_rhs: from the
// momentum values at tau (vm1, vm3 from B, vm2 from B*) and the z values (vz0; with zres, z is still in
// zbuf slot 6 from the R_z phase), u = m/rho, rho and C_ij = -m_i m_j/rho on the physical grid, u_hat by
// interpolation, T_ij = C_ij + tau_ij projected with the RHS of Omega2 and phi2 emitted at tau (eqs. om,
// phi with the body force), the Dirichlet / Neumann projections of the RHS (eq. mean_m1m3 for the means)
// and the RK2 update of phi2, Omega2 and the means (a->stage 0 or 1; 2: right-hand sides only).
static lmvd_status rhs_phase(const Ctx& c, const lmvd_substep_args* a, const double2* vz0, const double2* vm1,
                             const double2* vm2, const double2* vm3, bool zres) {
  lmvd_plan_s* p = c.p;
  const HostTables& H = p->H;
  const Workspace& W = p->ws;
  hipStream_t s = c.s;
  const size_t ncol = ncols(p);
  const size_t nB = ncol * H.n2;
  const bool xr = p->use_reg && xreg_size(H.cfg.m1, H.nl);
  double2* vals[kMaxOut];
  for (int g = 0; g < kMaxOut; ++g) vals[g] = c.at<double2>(W.off_vals[g]);
  double2* u[3];
  for (int i = 0; i < 3; ++i) u[i] = c.at<double2>(W.off_u[i]);
  double2* T[6];
  for (int i = 0; i < 6; ++i) T[i] = c.at<double2>(W.off_T[i]);
  double2* rhov = c.at<double2>(W.off_rhov);
  double2* vz1 = c.at<double2>(W.off_vz1);
  double2* vzl = c.at<double2>(W.off_vzl);
  double2* vz3 = c.at<double2>(W.off_vz3);
  double2* vmd1 = c.at<double2>(W.off_vmd1);
  double2* vmd3 = c.at<double2>(W.off_vmd3);
  double2* vc2d = c.at<double2>(W.off_vc2d);
  const double2* phi2 = static_cast<const double2*>(a->phi2);
  const double2* om2 = static_cast<const double2*>(a->omega2);
  lmvd_status st;
  double2* cv[6] = {vals[4], vals[5], vals[6], vals[7], vals[8], vals[9]};
  const std::vector<double2*> vel_out{vals[0], vals[1], vals[2], rhov, cv[0], cv[1], cv[2], cv[3], cv[4], cv[5]};
  if (zres) {  // z still in zbuf slot 6
    st = plane_phase<PH_VEL>(c, {ev(vm1, EV_IDENT), ev(vm2, EV_IDENT), ev(vm3, EV_IDENT)}, vel_out);
  } else if (xr) {
    EvalIn zin = ev(vz0, EV_IDENT);
    zin.slot = 6;
    st = plane_phase<PH_VEL>(c, {ev(vm1, EV_IDENT), ev(vm2, EV_IDENT), ev(vm3, EV_IDENT), zin}, vel_out);
  } else {
    st = plane_phase<PH_VEL>(c, {ev(vz0, EV_IDENT), ev(vm1, EV_IDENT), ev(vm2, EV_IDENT), ev(vm3, EV_IDENT)},
                             vel_out);
  }
  if (st != LMVD_OK) return st;
  {
    const int n = int(ncol);
    ProfScope ps(p, KC_PROJ, s, 3 * 4.0 * 16.0 * nB);
    col<JobProj3>(c, dim3((n + kThreads - 1) / kThreads, 3), 0, {0, ProjBatch{{vals[0], vals[1], vals[2]}, {u[0], u[1],
                  u[2]}}, n});
  }
  const bool narrow = H.p <= 8 && H.proj[0].lower <= 6 && H.proj[0].upper <= 6;
  const bool varmu = var_mu(H.cfg);
  if (varmu) {
    // mu = mu(z): tau_ij = mu(z) S_ij on the physical grid.  The S_ij values at tau come from u_hat and go
    // to the R_z inputs' buffers (dead by now).  Two physical passes, one per group of three components
    // (the two flux groups); z is still in zbuf slot 6 when all planes are one batch on the register
    // x-pass, else transformed again.  The tau_ij values land in T, which the flux kernels read and then
    // overwrite.
    double2* S[6] = {vz1, vzl, vz3, vmd1, vmd3, vc2d};
    {
      const int n = int(ncol);
      const dim3 grid((n + kThreads - 1) / kThreads);
      ProfScope ps(p, KC_FLUX, s, 16.0 * nB * 9.0);
      const SixPtr sp{{S[0], S[1], S[2], S[3], S[4], S[5]}};
      if (narrow) col<JobStrain<8>>(c, grid, 0, {u[0], u[1], u[2], sp});
      else col<JobStrain<kMaxW>>(c, grid, 0, {u[0], u[1], u[2], sp});
    }
    for (int grp = 0; grp < 2; ++grp) {
      std::vector<EvalIn> tin{ev(S[3 * grp], EV_IDENT), ev(S[3 * grp + 1], EV_IDENT), ev(S[3 * grp + 2], EV_IDENT)};
      if (!zres) {
        EvalIn zin = ev(vz0, EV_IDENT);
        if (xr) zin.slot = 6;  // the register x-pass reads z from slot 6, the generic one from slot 3
        tin.push_back(zin);
      }
      st = plane_phase<PH_TAU>(c, tin, {T[3 * grp], T[3 * grp + 1], T[3 * grp + 2]});
      if (st != LMVD_OK) return st;
    }
  }
  // fluxes and their share of the RHS values at tau (RO: Omega2, RP: phi2)
  double2* RO = vals[0];
  double2* RP = vals[1];
  {
    const int n = int(ncol);
    const dim3 grid((n + kThreads - 1) / kThreads);
    // per group: C_ij and u_hat (or tau_ij values) in, L-sweep intermediates out and back, RHS values out
    // (group 1 also reads them and rho)
    ProfScope ps(p, KC_FLUX, s, 16.0 * nB * 31.0);
    const FluxArgs fa{cv[0], cv[1], cv[2], u[0], u[1], u[2], T[0], T[1], T[2], RO, RP, rhov};
    const FluxArgs fb{cv[3], cv[4], cv[5], u[0], u[1], u[2], T[3], T[4], T[5], RO, RP, rhov};
    if (narrow && varmu) {
      col<JobFlux<0, 8, 6, true>>(c, grid, 0, fa);
      col<JobFlux<1, 8, 6, true>>(c, grid, 0, fb);
    } else if (narrow) {
      col<JobFlux<0, 8, 6>>(c, grid, 0, fa);
      col<JobFlux<1, 8, 6>>(c, grid, 0, fb);
    } else if (varmu) {
      col<JobFlux<0, kMaxW, kMaxBand, true>>(c, grid, 0, fa);
      col<JobFlux<1, kMaxW, kMaxBand, true>>(c, grid, 0, fb);
    } else {
      col<JobFlux<0, kMaxW, kMaxBand>>(c, grid, 0, fa);
      col<JobFlux<1, kMaxW, kMaxBand>>(c, grid, 0, fb);
    }
  }
  // RHS and RK2
  {
    const int n = int(ncol);
    {
      ProfScope ps(p, KC_RHS, s, 16.0 * nB * (a->stage ? 12.0 : 10.0) + 16.0 * nB * (a->rhs_phi2 ? 2 : 0));
      col<JobRhsFluct>(c, dim3((n + kThreads - 1) / kThreads), 0,
                       {RO, RP, phi2, om2, static_cast<const double2*>(a->rhs_phi2_prev),
                        static_cast<const double2*>(a->rhs_omega2_prev), static_cast<double2*>(a->phi2_out),
                        static_cast<double2*>(a->omega2_out), static_cast<double2*>(a->rhs_phi2),
                        static_cast<double2*>(a->rhs_omega2), c.at<double2>(W.off_yphi), c.at<double2>(W.off_yom),
                        a->stage});
    }
    {
      ProfScope ps(p, KC_RHS, s, 16.0 * 2 * H.n2 + 8.0 * H.n2 * (a->stage ? 8.0 : 6.0));
      col<JobRhsMean>(c, dim3(1), size_t(2) * H.n2 * sizeof(double),
                      {T[1], T[4], a->m1bar, a->m3bar, a->rhs_m1_prev, a->rhs_m3_prev, a->m1bar_out, a->m3bar_out,
                       a->rhs_m1, a->rhs_m3, a->stage});
    }
  }
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

// Fused m^c (k_mc) of one set of rho_t values at tau, on the workspace's two sweep scratch fields: V1, V2, V3
// receive the m^c values (V3 null: psi in V1, see mc_body); with d1..d3 the m^d values are added and rhoc, c2,
// mparc receive the coefficients.
static void launch_mc(const Ctx& c, const double2* vals, const double2* d1, const double2* d2, const double2* d3,
                      double2* V1, double2* V2, double2* V3, double2* rhoc, double2* c2, double2* mparc) {
  lmvd_plan_s* p = c.p;
  const HostTables& H = p->H;
  const int nth = 2 * H.nl * ((H.nn + 1) / 2);
  const dim3 g((nth + kThreads - 1) / kThreads);
  const bool narrow = H.proj[0].lower <= 6 && H.proj[0].upper <= 6;
  double2* yp = c.at<double2>(p->ws.off_yp);
  double2* yt = c.at<double2>(p->ws.off_yt);
  // the staged tables must leave room for two blocks per compute unit
  const McLds lay{H.n2, H.n2 + 1, narrow ? 6 : kMaxBand};
  const bool stage = lay.bytes() <= 72 * 1024;
#define LMVD_MC(LA_, LB_, ST_) \
  col<JobMc<LA_, LA_, LB_, ST_>>(c, g, ST_ ? lay.bytes() : 0, {vals, yp, yt, d1, d2, d3, V1, V2, V3, rhoc, c2, mparc})
  if (p->fac_la == 7 && narrow && stage)
    LMVD_MC(7, 6, true);
  else if (p->fac_la == 7 && narrow)
    LMVD_MC(7, 6, false);
  else if (p->fac_la == 7)
    LMVD_MC(7, kMaxBand, false);
  else
    LMVD_MC(8, kMaxBand, false);
#undef LMVD_MC
}

static lmvd_status run_substep(lmvd_plan_s* p, const lmvd_substep_args* a, void* workspace, hipStream_t s,
                               Recorder* rec = nullptr) {
  const HostTables& H = p->H;
  Ctx c{p, static_cast<char*>(workspace), s, rec};
  const Workspace& W = p->ws;
  const size_t ncol = ncols(p);
  const size_t nB = ncol * H.n2;
  const int kf = (a->kf < 0) ? H.cfg.kf : a->kf;
  double2* md1 = c.at<double2>(W.off_md1);
  double2* md3 = c.at<double2>(W.off_md3);
  double2* c2d = c.at<double2>(W.off_c2d);
  double2* mpar = c.at<double2>(W.off_mpar);
  double2* c2c = c.at<double2>(W.off_c2c);
  double2* rz = c.at<double2>(W.off_rz);
  double2* zta = c.at<double2>(W.off_zta);
  double2* ztb = c.at<double2>(W.off_ztb);
  double2* rhot = c.at<double2>(W.off_rhot);
  double2* vals[kMaxOut];
  for (int g = 0; g < kMaxOut; ++g) vals[g] = c.at<double2>(W.off_vals[g]);
  double2* u[3];
  for (int i = 0; i < 3; ++i) u[i] = c.at<double2>(W.off_u[i]);
  double2* T[6];
  for (int i = 0; i < 6; ++i) T[i] = c.at<double2>(W.off_T[i]);
  double2* rhov = c.at<double2>(W.off_rhov);
  const double2* z = static_cast<const double2*>(a->z);
  const double2* phi2 = static_cast<const double2*>(a->phi2);
  const double2* om2 = static_cast<const double2*>(a->omega2);
  double2* user_zt = static_cast<double2*>(a->zt);
  lmvd_status st;

  double2* vz0 = c.at<double2>(W.off_vz0);
  double2* vz1 = c.at<double2>(W.off_vz1);
  double2* vzl = c.at<double2>(W.off_vzl);
  double2* vz3 = c.at<double2>(W.off_vz3);
  double2* vmd1 = c.at<double2>(W.off_vmd1);
  double2* vmd3 = c.at<double2>(W.off_vmd3);
  double2* vc2d = c.at<double2>(W.off_vc2d);
  double2* vm1 = c.at<double2>(W.off_vm1c);
  double2* vm2 = c.at<double2>(W.off_vm2c);
  double2* vm3 = c.at<double2>(W.off_vm3c);
  double2* vzt = c.at<double2>(W.off_vzt);
  const dim3 cgrid((unsigned)((ncol + kThreads - 1) / kThreads));
  // m^c values (and, for the final iterate, m = m^d + m^c and the coefficients) from the rho_t values
  auto mc_step = [&](bool final_it) {
    // values in, L-sweep intermediate out and back, 2 value fields out (psi, m2; the final iterate 3), A(k)
    // sweep intermediate out and back, the factors once per pair; the final iterate also reads m^d values and
    // writes rho_t, m_par, c2
    const int nth = 2 * H.nl * ((H.nn + 1) / 2);
    ProfScope ps(p, KC_MC, s,
                 16.0 * nB * (final_it ? 11.0 : 5.0) + 16.0 * ncol * (H.n2 + 1) * (final_it ? 3.0 : 2.0) +
                     8.0 * H.fac_slots * (nth / 2));
    launch_mc(c, vals[0], final_it ? vmd1 : nullptr, final_it ? vc2d : nullptr, final_it ? vmd3 : nullptr, vm1, vm2,
              final_it ? vm3 : nullptr, final_it ? rhot : nullptr, final_it ? c2c : nullptr,
              final_it ? mpar : nullptr);
  };
  auto values = [&](const double2* a1, double2* v1, const double2* a2, double2* v2, const double2* a3, double2* v3) {
    ProfScope ps(p, KC_VALUES, s, 16.0 * nB * ((a1 ? 2 : 0) + (a2 ? 2 : 0) + (a3 ? 2 : 0)));
    (void)per_instance(c, [=](const Ctx& cc) {
      hipLaunchKernelGGL(k_values, cgrid, dim3(kThreads), 0, cc.s, cc.p->D, a1, v1, a2, v2, a3, v3);
      return LMVD_OK;
    });
  };

  // guess coefficients of the BDF-like extrapolation
  const double bn = H.cfg.beta_n, bp = H.cfg.beta_p;
  double co[4];
  if (a->stage == 0) {
    co[0] = 2.0; co[1] = -2.0 - 0.5 * bn; co[2] = bn; co[3] = -0.5 * bn;
  } else {
    co[0] = 4.0 + bp; co[1] = -5.0 - 2.0 * bp; co[2] = bp; co[3] = 1.0;
  }
  double2* gdst = (kf == 0 && user_zt) ? user_zt : zta;
  const int zero = (a->guess_mode == 1) ? 1 : 0;
  const ValuesZArgs zargs{z, vz0, vz1, vzl, vz3};
  const GuessArgs gargs{z, static_cast<const double2*>(a->z_hist[0]), static_cast<const double2*>(a->z_hist[1]),
                        static_cast<const double2*>(a->z_hist[2]), co[0], co[1], co[2], co[3], H.cfg.dt, zero,
                        gdst, vzt};
  // 1. m^d and its values at tau, the values of z (fixed during the substep) and the guess
  if (H.p == 8) {
    const int nth = 2 * H.nl * ((H.nn + 1) / 2);
    const bool diag = a->md[0] || a->md[1] || a->md[2];
    // m^d: phi2, Omega2 in, 3 value fields out, A(k) sweep intermediate out and back, factors once per
    // pair (+ the coefficients when requested); z values: 1 in, 4 out; guess: 4 (or 1) in, 2 out
    ProfScope ps(p, KC_MD, s,
                 16.0 * nB * (diag ? 7.0 : 5.0) + 16.0 * ncol * (H.n2 + 1) * (diag ? 3.0 : 2.0) +
                     8.0 * H.fac_slots * (nth / 2) + 16.0 * nB * 5 + 16.0 * nB * (zero ? 2 : 6));
    const dim3 g((unsigned(std::max<size_t>(nth, ncol)) + kThreads - 1) / kThreads, 3);
    const MdArgs margs{phi2, om2, a->m1bar, a->m3bar, c.at<double2>(W.off_yt), vmd1, vc2d, vmd3,
                       diag ? c2d : nullptr, diag ? md1 : nullptr, diag ? md3 : nullptr};
    if (p->fac_la == 7)
      col<JobPrologue<7, 7, 8>>(c, g, 0, {1, margs, zargs, gargs});
    else
      col<JobPrologue<8, 8, 8>>(c, g, 0, {1, margs, zargs, gargs});
  } else {
    (void)per_instance(c, [=](const Ctx& cc) {
      solveA<0>(cc, phi2, om2, a->m1bar, a->m3bar, c2d, md1, md3);
      return LMVD_OK;
    });
    values(md1, vmd1, md3, vmd3, c2d, vc2d);
    ProfScope ps(p, KC_VALUES, s, 16.0 * nB * 5 + 16.0 * nB * (zero ? 2 : 6));
    col<JobPrologue<8, 8, 8>>(c, dim3(cgrid.x, 2), 0, {0, MdArgs{}, zargs, gargs});
  }
  // 2. R_z
  // the register x-pass forms d z / d x from the z line and takes z from zbuf slot 6, where it stays for
  // the u, rho, C_ij pass when all planes are one batch; the generic x-pass takes them as inputs
  const bool xr = p->use_reg && xreg_size(H.cfg.m1, H.nl);
  {
    const std::vector<EvalIn> rin =
        xr ? std::vector<EvalIn>{ev(vzl, EV_IDENT), ev(vmd1, EV_IDENT), ev(vz1, EV_IDENT), ev(vc2d, EV_IDENT),
                                 ev(vz3, EV_IDENT), ev(vmd3, EV_IDENT), ev(vz0, EV_IDENT)}
           : std::vector<EvalIn>{ev(vzl, EV_IDENT), ev(vz0, EV_IDENT), ev(vz0, EV_IDENT, MU_IK1), ev(vmd1, EV_IDENT),
                                 ev(vz1, EV_IDENT), ev(vc2d, EV_IDENT), ev(vz3, EV_IDENT), ev(vmd3, EV_IDENT)};
    st = var_rhod(H.cfg) ? plane_phase<PH_RZV>(c, rin, {vals[0]}) : plane_phase<PH_RZ>(c, rin, {vals[0]});
  }
  if (st != LMVD_OK) return st;
  proj(c, 2, vals[0], rz);
  // The iterates before the last one are used only through their values at tau.  With all planes in
  // one batch and register z transforms, the L x-pass output is z-filtered (plus the filtered R_z
  // values, computed once here) in place of the forward transform, projection and inverse transform.
  const bool elide = p->pb == H.n2 && p->use_reg && zreg_size(H.cfg.m3) && kf >= 2 && W.off_szt != 0;
  double2* szt = c.at<double2>(W.off_szt);
  double2* zbuf0 = c.at<double2>(p->ws.off_zbuf);
  double2* obuf0 = c.at<double2>(p->ws.off_obuf);
  if (elide) zfilter(c, obuf0, nullptr, szt);
  if (kf == 0) {
    const double2* ztp = static_cast<const double2*>(a->zt_prev);
    double2* zo = static_cast<double2*>(a->z_out);
    const double dt = H.cfg.dt;
    const int stg = a->stage;
    (void)per_instance(c, [=](const Ctx& cc) {
      hipLaunchKernelGGL(k_zupdate, dim3((nB + kThreads - 1) / kThreads), dim3(kThreads), 0, cc.s, z, gdst, ztp, zo,
                         dt, stg, nB);
      return LMVD_OK;
    });
  }
  double2* cur = (kf == 0 && user_zt) ? user_zt : zta;
  // 3. fixed-point iterations z_t^k = L(z) z_t^{k-1} + R_z
  bool zt_filtered = false;  // the iterate's values are in zbuf already (z-filtered)
  for (int it = 0; it < kf; ++it) {
    const bool last = (it == kf - 1);
    st = plane_phase<PH_RHOT>(c, {ev(vzt, EV_IDENT)}, {vals[0]}, nullptr, nullptr, !zt_filtered);
    if (st != LMVD_OK) return st;
    mc_step(false);  // psi in vm1, m2 in vm2
    const bool filt = elide && !last;
    st = plane_phase<PH_L>(c, {ev(vm1, EV_IDENT, MU_IK1), ev(vm2, EV_IDENT), ev(vm1, EV_IDENT, MU_IK3)}, {vals[0]},
                           nullptr, nullptr, true, !filt);
    if (st != LMVD_OK) return st;
    zt_filtered = filt;
    if (filt) {
      zfilter(c, obuf0, szt, zbuf0);
      continue;
    }
    double2* next = (last && user_zt) ? user_zt : (cur == zta ? ztb : zta);
    const int n = int(ncol);
    const dim3 g((n + kThreads - 1) / kThreads);
    ProfScope ps(p, KC_PROJ_ZT, s, (last ? (a->stage ? 9.0 : 8.0) : 5.0) * 16.0 * nB);
    if (last)
      col<JobProj<EPI_ADD_ZUPDATE>>(c, g, 0,
                                    {2, vals[0], next, rz, z, static_cast<const double2*>(a->zt_prev),
                                     static_cast<double2*>(a->z_out), vzt, nullptr, a->stage, n});
    else
      col<JobProj<EPI_ADD>>(c, g, 0, {2, vals[0], next, rz, nullptr, nullptr, nullptr, vzt, nullptr, a->stage, n});
    cur = next;
  }
  // m^c of the stage from z_t^{k_f}
  st = plane_phase<PH_RHOT>(c, {ev(vzt, EV_IDENT)}, {vals[0]});
  if (st != LMVD_OK) return st;
  mc_step(true);  // m = m^d + m^c values
  // 4./5. velocities, density, fluxes, right-hand sides and the RK2 update
  st = rhs_phase(c, a, vz0, vm1, vm2, vm3, xr && p->pb == H.n2);
  if (st != LMVD_OK) return st;
  // optional diagnostics (never in a recorded substep)
  if (!rec) {
    const size_t sB = nB * 16, sS = ncol * (H.n2 + 1) * 16;
    if (a->md[0]) HIP_OK(hipMemcpyAsync(a->md[0], md1, sB, hipMemcpyDeviceToDevice, s));
    if (a->md[1]) HIP_OK(hipMemcpyAsync(a->md[1], c2d, sS, hipMemcpyDeviceToDevice, s));
    if (a->md[2]) HIP_OK(hipMemcpyAsync(a->md[2], md3, sB, hipMemcpyDeviceToDevice, s));
    if (a->mc[1]) HIP_OK(hipMemcpyAsync(a->mc[1], c2c, sS, hipMemcpyDeviceToDevice, s));
  }
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

__global__ void k_mc13(DevPlan P, const double2* __restrict__ mpar, double2* __restrict__ m1,
                       double2* __restrict__ m3) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ncol * P.n2) return;
  const size_t col = e % ncol;
  const int l = int(col % P.nl), ni = int(col / P.nl);
  const double k1 = P.k1[l], k3 = P.k3[ni];
  if (m1) m1[e] = apply_mult(MU_K1K, k1, k3, mpar[e]);
  if (m3) m3[e] = apply_mult(MU_K3K, k1, k3, mpar[e]);
}

static bool aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; }

}  // namespace lmvd

using namespace lmvd;

namespace lmvd {
// Argument checks of one substep (pointers present and aligned, stage and
// guess mode valid, the history and the stage's RHS buffers given).
static lmvd_status check_substep_args(lmvd_plan plan, const lmvd_substep_args* a, const void* workspace) {
  if (!plan || !a || !workspace) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (a->stage != 0 && a->stage != 1) return LMVD_EINVAL;
  if (a->guess_mode != 0 && a->guess_mode != 1) return LMVD_EINVAL;
  const void* req[] = {a->phi2, a->omega2, a->z, a->m1bar, a->m3bar, a->phi2_out, a->omega2_out, a->z_out,
                       a->m1bar_out, a->m3bar_out};
  for (const void* q : req)
    if (!q || !aligned(q)) return LMVD_EINVAL;
  if (a->z_out == a->z) return LMVD_EINVAL;
  if (a->stage == 0 && (!a->rhs_phi2 || !a->rhs_omega2 || !a->zt || !a->rhs_m1 || !a->rhs_m3)) return LMVD_EINVAL;
  if (a->stage == 1 && (!a->rhs_phi2_prev || !a->rhs_omega2_prev || !a->zt_prev || !a->rhs_m1_prev ||
                        !a->rhs_m3_prev))
    return LMVD_EINVAL;
  if (a->guess_mode == 0 && (!a->z_hist[0] || !a->z_hist[1] || !a->z_hist[2])) return LMVD_EINVAL;
  if (a->kf < -1 || a->kf > 10000) return LMVD_EINVAL;
  return LMVD_OK;
}
}  // namespace lmvd

extern "C" {

const char* lmvd_status_string(lmvd_status s) {
  switch (s) {
    case LMVD_OK: return "ok";
    case LMVD_EINVAL: return "invalid argument";
    case LMVD_ENOMEM: return "out of memory";
    case LMVD_EHIP: return "HIP error";
    case LMVD_EUNSUPPORTED: return "unsupported size";
    case LMVD_ENUMERIC: return "numerical failure (pivot)";
    case LMVD_ENONFINITE: return "non-finite value in the substep's outputs";
  }
  return "unknown status";
}

lmvd_status lmvd_plan_create(const lmvd_config* cfg, lmvd_plan* out) {
  std::string msg;
  lmvd_status st = create_plan(cfg, out, msg);
  if (st != LMVD_OK && !msg.empty()) fprintf(stderr, "lmvd_plan_create: %s\n", msg.c_str());
  return st;
}

lmvd_status lmvd_plan_destroy(lmvd_plan plan) {
  if (!plan) return LMVD_EINVAL;
  for (hipEvent_t e : plan->prof.ev) (void)hipEventDestroy(e);
  for (void* d : plan->allocs) (void)hipFree(d);
  delete plan;
  return LMVD_OK;
}

lmvd_status lmvd_sizes(lmvd_plan plan, size_t* se, size_t* ss, size_t* wb) {
  if (!plan) return LMVD_EINVAL;
  const size_t ncol = size_t(plan->H.nn) * plan->H.nl;
  if (se) *se = ncol * plan->H.n2;
  if (ss) *ss = ncol * (plan->H.n2 + 1);
  if (wb) *wb = plan->ws.bytes;
  return LMVD_OK;
}

namespace lmvd {
// non-finite scan of n doubles: one lane per wavefront that saw a NaN or an infinity sets the flag
__global__ void __launch_bounds__(kThreads) k_nonfinite(const double* __restrict__ x, size_t n, unsigned* flag) {
  bool bad = false;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__any(bad) && (threadIdx.x % 64) == 0) atomicOr(flag, 1u);
}
__global__ void k_clear_flag(unsigned* flag) {
  if (threadIdx.x == 0) flag[0] = 0u;
}
static lmvd_status scan_outputs(lmvd_plan_s* p, const lmvd_substep_args* a, hipStream_t s) {
  const size_t nS = 2 * size_t(p->H.nn) * p->H.nl * p->H.n2, n2 = size_t(p->H.n2);
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, s, p->finite_flag);
  const std::pair<const void*, size_t> f[] = {{a->z_out, nS}, {a->phi2_out, nS}, {a->omega2_out, nS},
                                              {a->m1bar_out, n2}, {a->m3bar_out, n2}, {a->zt, nS}};
  for (const auto& q : f)
    if (q.first)
      hipLaunchKernelGGL(k_nonfinite, dim3(1024), dim3(kThreads), 0, s, static_cast<const double*>(q.first),
                         q.second, p->finite_flag);
  unsigned h = 0;
  if (hipMemcpyAsync(&h, p->finite_flag, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return LMVD_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return LMVD_EHIP;
  return h ? LMVD_ENONFINITE : LMVD_OK;
}
}  // namespace lmvd

lmvd_status lmvd_substep(lmvd_plan plan, const lmvd_substep_args* a, void* workspace, void* stream) {
  const lmvd_status ck = lmvd::check_substep_args(plan, a, workspace);
  if (ck != LMVD_OK) return ck;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lmvd_status st = run_substep(plan, a, workspace, s);
  if (st != LMVD_OK) return st;
  if (a->mc[0] || a->mc[2]) {
    const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
    hipLaunchKernelGGL(k_mc13, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, plan->D,
                       reinterpret_cast<const double2*>(static_cast<char*>(workspace) + plan->ws.off_mpar),
                       static_cast<double2*>(a->mc[0]), static_cast<double2*>(a->mc[2]));
  }
  if (hipGetLastError() != hipSuccess) return LMVD_EHIP;
  if (plan->H.cfg.check_finite) return lmvd::scan_outputs(plan, a, s);
  return LMVD_OK;
}

lmvd_status lmvd_substep_noalloc(lmvd_plan plan, const lmvd_substep_args* a, void* stream) {
  if (!plan || !a) return LMVD_EINVAL;
  if (plan->ws.bytes > lmvd::kNoAllocBytes) return LMVD_EUNSUPPORTED;
  void* ws = lmvd::device_scratch(plan->device);
  if (!ws) return LMVD_EHIP;
  return lmvd_substep(plan, a, ws, stream);
}

lmvd_status lmvd_noalloc_capacity(size_t* bytes) {
  if (!bytes) return LMVD_EINVAL;
  *bytes = lmvd::kNoAllocBytes;
  return LMVD_OK;
}

struct lmvd_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* arena = nullptr;  // plans and job records of the grouped launches
  int device = 0;
  int grouped = 0;
};

namespace lmvd {
// Capture of count instances x nsub substeps on `origin`.  Grouped: every
// column job is one launch over all instances (records in `arena`), and the
// per-instance work between them (plane phases) runs on one branch stream per
// instance.  Used when all instances record the same sequence of jobs (same
// k_f, stage pattern and kernel variants); otherwise every instance is one
// branch of its own.
static lmvd_status capture_graph(const lmvd_plan* plans, const lmvd_substep_args* args, void* const* workspaces,
                                 int count, int nsub, hipStream_t origin, std::vector<hipStream_t>& br,
                                 std::vector<hipEvent_t>& ev, lmvd_graph_s* g) {
  std::vector<Recorder> rec(count);
  for (int i = 0; i < count; ++i)
    for (int k = 0; k < nsub; ++k) {
      const lmvd_status st = run_substep(plans[i], &args[size_t(i) * nsub + k], workspaces[i], nullptr, &rec[i]);
      if (st != LMVD_OK) return st;
    }
  const size_t nops = rec[0].ops.size();
  bool same = true;
  for (int i = 1; i < count && same; ++i) {
    if (rec[i].ops.size() != nops) {
      same = false;
      break;
    }
    for (size_t j = 0; j < nops && same; ++j) {
      const RecOp &x = rec[0].ops[j], &y = rec[i].ops[j];
      if ((x.job == nullptr) != (y.job == nullptr)) same = false;
    }
  }
  auto fail_capture = [&](lmvd_status e) {
    hipGraph_t junk = nullptr;
    if (hipStreamEndCapture(origin, &junk) == hipSuccess && junk) (void)hipGraphDestroy(junk);
    return e;
  };
  if (!same) {
    // one branch per instance, its substeps in order
    if (hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal) != hipSuccess) return LMVD_EHIP;
    if (hipEventRecord(ev[count], origin) != hipSuccess) return fail_capture(LMVD_EHIP);
    for (int i = 0; i < count; ++i) {
      if (hipStreamWaitEvent(br[i], ev[count], 0) != hipSuccess) return fail_capture(LMVD_EHIP);
      for (int k = 0; k < nsub; ++k) {
        const lmvd_status st = run_substep(plans[i], &args[size_t(i) * nsub + k], workspaces[i], br[i]);
        if (st != LMVD_OK) return fail_capture(st);
      }
      if (hipEventRecord(ev[i], br[i]) != hipSuccess || hipStreamWaitEvent(origin, ev[i], 0) != hipSuccess)
        return fail_capture(LMVD_EHIP);
    }
    if (hipStreamEndCapture(origin, &g->graph) != hipSuccess) return LMVD_EHIP;
    g->grouped = 0;
    return LMVD_OK;
  }
  // arena: the instances' plans, then for each job op and each distinct job at it (instances of different
  // sizes run different kernels) the records of the instances that run it
  struct Launch {
    const JobOps* job;
    size_t off;
    int n;
    unsigned blocks;
    size_t lds;
  };
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  std::vector<unsigned char> host(al(size_t(count) * sizeof(DevPlan)));
  for (int i = 0; i < count; ++i) std::memcpy(host.data() + size_t(i) * sizeof(DevPlan), &plans[i]->D, sizeof(DevPlan));
  std::vector<std::vector<Launch>> launches(nops);
  for (size_t j = 0; j < nops; ++j) {
    if (!rec[0].ops[j].job) continue;
    std::vector<const JobOps*> seen;
    for (int i = 0; i < count; ++i) {
      const JobOps* job = rec[i].ops[j].job;
      if (std::find(seen.begin(), seen.end(), job) != seen.end()) continue;
      seen.push_back(job);
      Launch L{job, host.size(), 0, 0, 0};
      for (int q = i; q < count; ++q) {
        const RecOp& o = rec[q].ops[j];
        if (o.job != job) continue;
        host.resize(L.off + size_t(L.n + 1) * job->rec_size);
        job->pack(host.data() + L.off + size_t(L.n) * job->rec_size, o.args.data(), q, L.blocks, o.grid);
        L.blocks += o.grid.x * o.grid.y * o.grid.z;
        L.lds = std::max(L.lds, o.lds);
        ++L.n;
      }
      host.resize(al(host.size()));
      launches[j].push_back(L);
    }
  }
  if (hipMalloc(&g->arena, host.size()) != hipSuccess) return LMVD_ENOMEM;
  if (hipMemcpy(g->arena, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) return LMVD_EHIP;
  const char* dev = static_cast<const char*>(g->arena);
  const DevPlan* dplans = reinterpret_cast<const DevPlan*>(dev);
  if (hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal) != hipSuccess) return LMVD_EHIP;
  for (size_t j = 0; j < nops;) {
    if (rec[0].ops[j].job) {
      const std::vector<Launch>& LS = launches[j];
      if (LS.size() == 1) {
        LS[0].job->launch(dplans, dev + LS[0].off, LS[0].n, LS[0].blocks, LS[0].lds, origin);
      } else {
        // the launches of one step cover disjoint instances: side by side on branch streams
        if (hipEventRecord(ev[count], origin) != hipSuccess) return fail_capture(LMVD_EHIP);
        for (size_t k = 0; k < LS.size(); ++k) {
          if (hipStreamWaitEvent(br[k], ev[count], 0) != hipSuccess) return fail_capture(LMVD_EHIP);
          LS[k].job->launch(dplans, dev + LS[k].off, LS[k].n, LS[k].blocks, LS[k].lds, br[k]);
          if (hipEventRecord(ev[k], br[k]) != hipSuccess || hipStreamWaitEvent(origin, ev[k], 0) != hipSuccess)
            return fail_capture(LMVD_EHIP);
        }
      }
      ++j;
      continue;
    }
    size_t j2 = j;  // a run of per-instance work: one branch per instance
    while (j2 < nops && !rec[0].ops[j2].job) ++j2;
    if (hipEventRecord(ev[count], origin) != hipSuccess) return fail_capture(LMVD_EHIP);
    for (int i = 0; i < count; ++i) {
      if (hipStreamWaitEvent(br[i], ev[count], 0) != hipSuccess) return fail_capture(LMVD_EHIP);
      for (size_t q = j; q < j2; ++q) {
        const lmvd_status st = rec[i].ops[q].fn(br[i]);
        if (st != LMVD_OK) return fail_capture(st);
      }
      if (hipEventRecord(ev[i], br[i]) != hipSuccess || hipStreamWaitEvent(origin, ev[i], 0) != hipSuccess)
        return fail_capture(LMVD_EHIP);
    }
    j = j2;
  }
  if (hipGetLastError() != hipSuccess) return fail_capture(LMVD_EHIP);
  if (hipStreamEndCapture(origin, &g->graph) != hipSuccess) return LMVD_EHIP;
  g->grouped = 1;
  return LMVD_OK;
}
}  // namespace lmvd

lmvd_status lmvd_graph_create(const lmvd_plan* plans, const lmvd_substep_args* args, void* const* workspaces,
                              int32_t count, int32_t nsub, lmvd_graph* out) {
  if (!plans || !args || !workspaces || !out || count < 1 || nsub < 1) return LMVD_EINVAL;
  *out = nullptr;
  const int dev = plans[0] ? plans[0]->device : 0;
  for (int i = 0; i < count; ++i) {
    lmvd_plan p = plans[i];
    if (!p || p->device != dev || p->prof.cls >= 0 || p->H.cfg.check_finite) return LMVD_EINVAL;
    for (int k = 0; k < nsub; ++k) {
      const lmvd_substep_args* a = &args[size_t(i) * nsub + k];
      const lmvd_status ck = lmvd::check_substep_args(p, a, workspaces[i]);
      if (ck != LMVD_OK) return ck;
      for (int q = 0; q < 3; ++q)
        if (a->md[q] || a->mc[q]) return LMVD_EINVAL;
    }
  }
  if (hipSetDevice(dev) != hipSuccess) return LMVD_EHIP;
  lmvd_graph g = new (std::nothrow) lmvd_graph_s;
  if (!g) return LMVD_ENOMEM;
  g->device = dev;
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> br(count, nullptr);
  std::vector<hipEvent_t> ev(count + 1, nullptr);
  lmvd_status st = LMVD_OK;
  if (hipStreamCreateWithFlags(&origin, hipStreamNonBlocking) != hipSuccess) st = LMVD_EHIP;
  for (int i = 0; i < count && st == LMVD_OK; ++i)
    if (hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) st = LMVD_EHIP;
  for (int i = 0; i <= count && st == LMVD_OK; ++i)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) st = LMVD_EHIP;
  if (st == LMVD_OK) st = lmvd::capture_graph(plans, args, workspaces, count, nsub, origin, br, ev, g);
  if (st == LMVD_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) st = LMVD_EHIP;
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t b : br)
    if (b) (void)hipStreamDestroy(b);
  if (origin) (void)hipStreamDestroy(origin);
  if (st != LMVD_OK) {
    (void)lmvd_graph_destroy(g);
    return st;
  }
  *out = g;
  return LMVD_OK;
}

lmvd_status lmvd_graph_launch(lmvd_graph g, void* stream) {
  if (!g || !g->exec) return LMVD_EINVAL;
  if (hipSetDevice(g->device) != hipSuccess) return LMVD_EHIP;
  return hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_graph_grouped(lmvd_graph g, int32_t* grouped) {
  if (!g || !grouped) return LMVD_EINVAL;
  *grouped = g->grouped;
  return LMVD_OK;
}

lmvd_status lmvd_graph_destroy(lmvd_graph g) {
  if (!g) return LMVD_EINVAL;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->arena) (void)hipFree(g->arena);
  delete g;
  return LMVD_OK;
}

lmvd_status lmvd_graph_autotune(const lmvd_plan* plans, const lmvd_substep_args* args, void* const* workspaces,
                                int32_t count, int32_t nsub, void* stream, int32_t launches, int32_t* zdivs,
                                double* ms_per_launch) {
  if (!plans || !args || !workspaces || count < 1 || nsub < 1 || launches < 1 || launches > 100)
    return LMVD_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return LMVD_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (hipSetDevice(plans[0]->device) != hipSuccess) return LMVD_EHIP;
  auto tileable = [](lmvd_plan p) { return p->use_reg && zreg_size(p->H.cfg.m3) && p->H.cfg.m3 != 768; };
  std::vector<int> sizes;
  for (int i = 0; i < count; ++i) {
    if (!tileable(plans[i])) continue;
    plans[i]->zdiv = 1;
    if (std::find(sizes.begin(), sizes.end(), plans[i]->H.cfg.m3) == sizes.end()) sizes.push_back(plans[i]->H.cfg.m3);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return LMVD_EHIP;
  }
  // one measurement: capture the graph with the current tiles, one warm-up launch, then `launches` timed
  auto measure = [&](double& ms) -> lmvd_status {
    lmvd_graph g = nullptr;
    lmvd_status st = lmvd_graph_create(plans, args, workspaces, count, nsub, &g);
    if (st != LMVD_OK) return st;
    st = lmvd_graph_launch(g, stream);
    if (st == LMVD_OK && hipEventRecord(e0, s) != hipSuccess) st = LMVD_EHIP;
    for (int r = 0; r < launches && st == LMVD_OK; ++r) st = lmvd_graph_launch(g, stream);
    float t = 0.0f;
    if (st == LMVD_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      st = LMVD_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess && st == LMVD_OK) st = LMVD_EHIP;
    (void)lmvd_graph_destroy(g);
    ms = double(t) / launches;
    return st;
  };
  double best = 0.0;
  lmvd_status st = measure(best);
  // coordinate descent over the transform sizes present: one tile code per size (line plan and divisor),
  // kept when it is at least 1 % faster than the best so far
  for (size_t k = 0; k < sizes.size() && st == LMVD_OK; ++k) {
    int cur = 1;
    std::vector<int> codes;
    for (int v = 0; v < zplan_count(sizes[k]); ++v)
      for (int dd : {1, 2, 4})
        if (dd + 8 * v != 1) codes.push_back(dd + 8 * v);
    for (int d : codes) {
      for (int i = 0; i < count; ++i)
        if (tileable(plans[i]) && plans[i]->H.cfg.m3 == sizes[k]) plans[i]->zdiv = d;
      double t = 0.0;
      st = measure(t);
      if (st != LMVD_OK) break;
      if (t < 0.99 * best) {
        best = t;
        cur = d;
      }
    }
    for (int i = 0; i < count; ++i)
      if (tileable(plans[i]) && plans[i]->H.cfg.m3 == sizes[k]) plans[i]->zdiv = cur;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (zdivs)
    for (int i = 0; i < count; ++i) zdivs[i] = plans[i]->zdiv;
  if (ms_per_launch) *ms_per_launch = best;
  return st;
}

lmvd_status lmvd_autotune(lmvd_plan plan, void* workspace, void* stream, int32_t force, int32_t* zdiv,
                          double* times_ms) {
  if (!plan || !workspace || !zdiv) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (force != 0 && !ztile_valid(force)) return LMVD_EINVAL;
  if (plan->prof.cls >= 0) return LMVD_EINVAL;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  const HostTables& H = plan->H;
  const int M3 = H.cfg.m3;
  const int cand[9] = {1, 2, 4, 9, 10, 12, 17, 18, 20};
  const int ncand = 3 * zplan_count(M3);
  if (times_ms)
    for (int i = 0; i < 9; ++i) times_ms[i] = -1.0;
  // only the register z kernels below 768 points have a tile choice
  if (!(plan->use_reg && zreg_size(M3) && M3 != 768)) {
    plan->zdiv = 1;
    *zdiv = 1;
    return LMVD_OK;
  }
  if (force) {
    plan->zdiv = force;
    *zdiv = force;
    return LMVD_OK;
  }
  // time the inverse and forward z transforms of three fields over the plan's plane batch, on the
  // workspace's own value and staging buffers (their contents do not matter for the timing)
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ctx c{plan, static_cast<char*>(workspace), s};
  const Workspace& W = plan->ws;
  EvalArgs A{};
  OutPtrs V{};
  for (int f = 0; f < 3; ++f) {
    A.in[f] = ev(c.at<double2>(W.off_vals[f]), EV_IDENT);
    A.in[f].slot = f;
    V.v[f] = c.at<double2>(W.off_vals[3 + f]);
  }
  double2* zbuf = c.at<double2>(W.off_zbuf);
  double2* obuf = c.at<double2>(W.off_obuf);
  const int nb = std::min(plan->pb, H.n2);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LMVD_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LMVD_EHIP;
  }
  const int saved = plan->zdiv;
  int best = 1;
  float best_ms = 0.0f;
  lmvd_status st = LMVD_OK;
  for (int i = 0; i < ncand && st == LMVD_OK; ++i) {
    plan->zdiv = cand[i];
    auto pass = [&]() {
#define CALLZ(N) launch_zinv_t<N>(c, A, zbuf, 0, nb, 3)
      LMVD_ZSWITCH(M3, CALLZ)
#undef CALLZ
#define CALLF(N) launch_zfwd_t<N>(c, obuf, V, 0, nb, 3)
      LMVD_ZSWITCH(M3, CALLF)
#undef CALLF
    };
    pass();  // warm-up
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess) st = LMVD_EHIP;
    for (int r = 0; r < 5 && st == LMVD_OK; ++r) pass();
    if (st == LMVD_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = LMVD_EHIP;
    if (st == LMVD_OK && hipGetLastError() != hipSuccess) st = LMVD_EHIP;
    if (times_ms) times_ms[i] = ms / 5.0;
    if (i == 0 || ms < best_ms) {
      best = cand[i];
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->zdiv = (st == LMVD_OK) ? best : saved;
  *zdiv = plan->zdiv;
  return st;
}

lmvd_status lmvd_to_physical(lmvd_plan plan, const void* values, double* phys, void* workspace, void* stream) {
  if (!plan || !values || !phys || !workspace) return LMVD_EINVAL;
  Ctx c{plan, static_cast<char*>(workspace), static_cast<hipStream_t>(stream)};
  return plane_phase<PH_TOPHYS>(c, {ev(values, EV_IDENT)}, {}, phys, nullptr);
}

lmvd_status lmvd_to_spectral(lmvd_plan plan, const double* phys, void* values, void* workspace, void* stream) {
  if (!plan || !values || !phys || !workspace) return LMVD_EINVAL;
  Ctx c{plan, static_cast<char*>(workspace), static_cast<hipStream_t>(stream)};
  return plane_phase<PH_FROMPHYS>(c, {}, {static_cast<double2*>(values)}, nullptr, phys);
}

lmvd_status lmvd_project(lmvd_plan plan, int32_t kind, const void* values, void* coeffs, void* stream) {
  if (!plan || !values || !coeffs || kind < 0 || kind > 2) return LMVD_EINVAL;
  Ctx c{plan, nullptr, static_cast<hipStream_t>(stream)};
  proj(c, kind, static_cast<const double2*>(values), static_cast<double2*>(coeffs));
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_evaluate(lmvd_plan plan, int32_t deriv, int32_t star, const void* coeffs, void* values,
                          void* stream) {
  if (!plan || !coeffs || !values || deriv < 0 || deriv > 2 || (star && deriv != 0)) return LMVD_EINVAL;
  const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
  const int kind = star ? EV_F0 : deriv;
  hipLaunchKernelGGL(k_evaluate, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), plan->D, kind, static_cast<const double2*>(coeffs),
                     static_cast<double2*>(values));
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_evaluate_adjoint(lmvd_plan plan, int32_t deriv, int32_t star, const void* values, void* coeffs,
                                  void* stream) {
  if (!plan || !values || !coeffs || deriv < 0 || deriv > 2 || (star && deriv != 0) || values == coeffs)
    return LMVD_EINVAL;
  const size_t ncol = size_t(plan->H.nn) * plan->H.nl;
  const int rows = star ? plan->H.n2 + 1 : plan->H.n2;
  hipLaunchKernelGGL(k_evaluate_t, dim3(unsigned((ncol + kThreads - 1) / kThreads), unsigned(rows)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), plan->D, star ? int(EV_F0) : deriv,
                     static_cast<const double2*>(values), static_cast<double2*>(coeffs));
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_project_adjoint(lmvd_plan plan, int32_t kind, const void* coeffs, void* values, void* stream) {
  if (!plan || !coeffs || !values || kind < 0 || kind > 2 || coeffs == values) return LMVD_EINVAL;
  const size_t ncol = size_t(plan->H.nn) * plan->H.nl;
  ProjTJobs J{};
  J.in[0] = static_cast<const double2*>(coeffs);
  J.out[0] = static_cast<double2*>(values);
  hipLaunchKernelGGL(k_project_t, dim3((ncol + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), plan->D, int(kind), J);
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_md_adjoint(lmvd_plan plan, const void* m1, const void* m2, const void* m3, void* phi2,
                           void* omega2, double* m1bar, double* m3bar, void* workspace, void* stream) {
  if (!plan || !m1 || !m2 || !m3 || !phi2 || !omega2 || !m1bar || !m3bar || !workspace) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t ncol = size_t(plan->H.nn) * plan->H.nl;
  double2* scr = reinterpret_cast<double2*>(static_cast<char*>(workspace) + plan->ws.off_yt);
  hipLaunchKernelGGL(k_md_t, dim3((ncol + kThreads - 1) / kThreads), dim3(kThreads), 0, s, plan->D,
                     static_cast<const double2*>(m1), static_cast<const double2*>(m2),
                     static_cast<const double2*>(m3), static_cast<double2*>(phi2), static_cast<double2*>(omega2),
                     m1bar, m3bar, scr);
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_mc_adjoint(lmvd_plan plan, const void* m1, const void* m2, const void* m3, void* rhot,
                           void* workspace, void* stream) {
  if (!plan || !m1 || !m2 || !m3 || !rhot || !workspace) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t ncol = size_t(plan->H.nn) * plan->H.nl;
  double2* scr = reinterpret_cast<double2*>(static_cast<char*>(workspace) + plan->ws.off_yt);
  hipLaunchKernelGGL(k_mc_t, dim3((ncol + kThreads - 1) / kThreads), dim3(kThreads), 0, s, plan->D,
                     static_cast<const double2*>(m1), static_cast<const double2*>(m2),
                     static_cast<const double2*>(m3), static_cast<double2*>(rhot), scr);
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_to_physical_adjoint(lmvd_plan plan, const double* phys, void* values, void* workspace,
                                     void* stream) {
  const lmvd_status st = lmvd_to_spectral(plan, phys, values, workspace, stream);
  if (st != LMVD_OK) return st;
  const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
  hipLaunchKernelGGL(k_scale_modes, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), plan->D, static_cast<const double2*>(values),
                     static_cast<double2*>(values), 0);
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_to_spectral_adjoint(lmvd_plan plan, const void* values, double* phys, void* workspace,
                                     void* stream) {
  if (!plan || !values || !phys || !workspace) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  // the scaled copy goes to a value field of the workspace that the inverse transform does not use
  double2* tmp = reinterpret_cast<double2*>(static_cast<char*>(workspace) + plan->ws.off_vals[kMaxOut - 1]);
  const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
  hipLaunchKernelGGL(k_scale_modes, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     static_cast<hipStream_t>(stream), plan->D, static_cast<const double2*>(values), tmp, 1);
  if (hipGetLastError() != hipSuccess) return LMVD_EHIP;
  return lmvd_to_physical(plan, tmp, phys, workspace, stream);
}

lmvd_status lmvd_rhs(lmvd_plan plan, const void* z, const void* m1, const void* m2, const void* m3, void* rhs_phi2,
                     void* rhs_omega2, double* rhs_m1, double* rhs_m3, void* workspace, void* stream) {
  if (!plan || !z || !m1 || !m2 || !m3 || !rhs_phi2 || !rhs_omega2 || !rhs_m1 || !rhs_m3 || !workspace)
    return LMVD_EINVAL;
  for (const void* q : {z, m1, m2, m3, static_cast<const void*>(rhs_phi2), static_cast<const void*>(rhs_omega2),
                        static_cast<const void*>(rhs_m1), static_cast<const void*>(rhs_m3)})
    if (!aligned(q)) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ctx c{plan, static_cast<char*>(workspace), s};
  const Workspace& W = plan->ws;
  double2* vz0 = c.at<double2>(W.off_vz0);
  double2* vm[3] = {c.at<double2>(W.off_vm1c), c.at<double2>(W.off_vm2c), c.at<double2>(W.off_vm3c)};
  const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
  const dim3 g((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_evaluate, g, dim3(kThreads), 0, s, plan->D, int(EV_E0), static_cast<const double2*>(z), vz0);
  hipLaunchKernelGGL(k_evaluate, g, dim3(kThreads), 0, s, plan->D, int(EV_E0), static_cast<const double2*>(m1), vm[0]);
  hipLaunchKernelGGL(k_evaluate, g, dim3(kThreads), 0, s, plan->D, int(EV_F0), static_cast<const double2*>(m2), vm[1]);
  hipLaunchKernelGGL(k_evaluate, g, dim3(kThreads), 0, s, plan->D, int(EV_E0), static_cast<const double2*>(m3), vm[2]);
  lmvd_substep_args a{};
  a.stage = 2;  // right-hand sides only
  a.rhs_phi2 = rhs_phi2;
  a.rhs_omega2 = rhs_omega2;
  a.rhs_m1 = rhs_m1;
  a.rhs_m3 = rhs_m3;
  return rhs_phase(c, &a, vz0, vm[0], vm[1], vm[2], false);
}

lmvd_status lmvd_md(lmvd_plan plan, const void* phi2, const void* omega2, const double* m1bar, const double* m3bar,
                    void* m1, void* m2, void* m3, void* workspace, void* stream) {
  if (!plan || !phi2 || !omega2 || !m1bar || !m3bar || !m1 || !m2 || !m3 || !workspace) return LMVD_EINVAL;
  Ctx c{plan, static_cast<char*>(workspace), static_cast<hipStream_t>(stream)};
  solveA<0>(c, static_cast<const double2*>(phi2), static_cast<const double2*>(omega2), m1bar, m3bar,
            static_cast<double2*>(m2), static_cast<double2*>(m1), static_cast<double2*>(m3));
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_mc(lmvd_plan plan, const void* rhot, void* m1, void* m2, void* m3, void* workspace, void* stream) {
  if (!plan || !rhot || !m1 || !m2 || !m3 || !workspace) return LMVD_EINVAL;
  Ctx c{plan, static_cast<char*>(workspace), static_cast<hipStream_t>(stream)};
  double2* mpar = c.at<double2>(plan->ws.off_mpar);
  solveA<1>(c, static_cast<const double2*>(rhot), nullptr, nullptr, nullptr, static_cast<double2*>(m2), mpar,
            nullptr);
  const size_t n = size_t(plan->H.nn) * plan->H.nl * plan->H.n2;
  hipLaunchKernelGGL(k_mc13, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, c.s, plan->D, mpar,
                     static_cast<double2*>(m1), static_cast<double2*>(m3));
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

lmvd_status lmvd_profile_start(lmvd_plan plan, int32_t cls, int32_t max_launches) {
  if (!plan || cls < 0 || cls >= KC_COUNT || max_launches < 1 || max_launches > (1 << 20)) return LMVD_EINVAL;
  lmvd_prof& f = plan->prof;
  for (hipEvent_t e : f.ev) (void)hipEventDestroy(e);
  f.ev.assign(size_t(2) * max_launches, nullptr);
  for (auto& e : f.ev)
    if (hipEventCreate(&e) != hipSuccess) return LMVD_EHIP;
  f.used = 0;
  f.bytes = 0.0;
  f.cls = cls;
  return LMVD_OK;
}

lmvd_status lmvd_profile_stop(lmvd_plan plan, double* total_ms, int64_t* launches, double* compulsory_bytes) {
  if (!plan) return LMVD_EINVAL;
  lmvd_prof& f = plan->prof;
  double tot = 0.0;
  for (int i = 0; i < f.used; ++i) {
    if (hipEventSynchronize(f.ev[2 * i + 1]) != hipSuccess) return LMVD_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, f.ev[2 * i], f.ev[2 * i + 1]) != hipSuccess) return LMVD_EHIP;
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = f.used;
  if (compulsory_bytes) *compulsory_bytes = f.bytes;
  for (hipEvent_t e : f.ev) (void)hipEventDestroy(e);
  f.ev.clear();
  f.cls = -1;
  f.used = 0;
  return LMVD_OK;
}

lmvd_status lmvd_factor_check(lmvd_plan plan, double growth_max, double* max_growth, double* min_pivot_ratio,
                              int64_t* bad_rows) {
  if (!plan || !(growth_max >= 0.0)) return LMVD_EINVAL;
  if (growth_max > 0.0) {
    if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
    const lmvd_status st = lmvd::factor_and_check(plan, growth_max);
    if (st != LMVD_OK && st != LMVD_ENUMERIC) return st;
  }
  if (max_growth) *max_growth = plan->fac_growth;
  if (min_pivot_ratio) *min_pivot_ratio = plan->fac_pivot;
  if (bad_rows) *bad_rows = plan->fac_bad;
  return plan->fac_bad ? LMVD_ENUMERIC : LMVD_OK;
}

lmvd_status lmvd_factor_check_host(const lmvd_config* cfg, double growth_max, double* max_growth,
                                   double* min_pivot_ratio, int64_t* bad_rows, int64_t* distinct_k) {
  if (!cfg || !(growth_max > 0.0)) return LMVD_EINVAL;
  HostTables H;
  std::string msg;
  lmvd_status st = build_host_tables(*cfg, H, msg);
  if (st != LMVD_OK) return st;
  FactorCheck fc;
  st = factor_check_host(H, growth_max, fc);
  if (max_growth) *max_growth = fc.max_growth;
  if (min_pivot_ratio) *min_pivot_ratio = fc.min_pivot_ratio;
  if (bad_rows) *bad_rows = fc.bad_rows;
  if (distinct_k) *distinct_k = fc.distinct_k;
  return st;
}

lmvd_status lmvd_basis_values(const lmvd_config* cfg, int32_t npts, const double* y, int32_t star, double* out) {
  if (!cfg || npts < 0 || (npts > 0 && (!y || !out)) || (star != 0 && star != 1)) return LMVD_EINVAL;
  HostTables H;
  std::string msg;
  lmvd_status st = build_host_tables(*cfg, H, msg);
  if (st != LMVD_OK) return st;
  std::vector<double> v;
  st = basis_values(H, star, std::vector<double>(y, y + npts), v);
  if (st != LMVD_OK) return st;
  std::copy(v.begin(), v.end(), out);
  return LMVD_OK;
}

lmvd_status lmvd_host_tables(const lmvd_config* cfg, double* tau, double* tau_star, double* E0, double* E1,
                             double* E2) {
  if (!cfg) return LMVD_EINVAL;
  HostTables H;
  std::string msg;
  lmvd_status st = build_host_tables(*cfg, H, msg);
  if (st != LMVD_OK) return st;
  if (tau) std::copy(H.tau.begin(), H.tau.end(), tau);
  if (tau_star) std::copy(H.tau_s.begin(), H.tau_s.end(), tau_star);
  double* outs[3] = {E0, E1, E2};
  for (int d = 0; d < 3; ++d)
    if (outs[d]) {
      std::vector<double> D = dense(H.E[d]);
      std::copy(D.begin(), D.end(), outs[d]);
    }
  return LMVD_OK;
}

}  // extern "C"

#include "substep_adjoint.h"
