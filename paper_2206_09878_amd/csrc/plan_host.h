// Host-side tables of the y-discretisation and the x-z transforms.
//
// Everything here runs on the CPU at plan creation; the device kernels read
// the uploaded copies.  B-splines (App. C of the paper): order p on clamped
// knots for every field except m2, order p+1 for m2; collocation at the
// Greville abscissae.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lmvd.h"

namespace lmvd {

constexpr int kMaxW = 10;       // nonzeros of one collocation row (order <= 9 -> <= 10)
constexpr int kMaxBand = 9;     // half-bandwidth limit of the no-pivot LU tables
constexpr int kMaxStages = 12;  // FFT passes

// A banded row table: row i has nonzeros in columns lo[i] .. lo[i]+kMaxW-1
// (zero-padded); w[i*kMaxW + q] multiplies column lo[i]+q.
struct RowTable {
  std::vector<int32_t> lo;
  std::vector<double> w;
  int rows = 0;
  int cols = 0;
  double at(int i, int j) const {
    int q = j - lo[i];
    return (q >= 0 && q < kMaxW) ? w[size_t(i) * kMaxW + q] : 0.0;
  }
};

// No-pivot banded LU of a shared (k-independent) matrix: row i of L has
// multipliers lmul[i*kMaxBand + (m-1)] for row i-m (m = 1..lower), row i of
// U has entries u[i*(kMaxBand+1) + q] for column i+q (q = 1..upper) and
// uinv[i] = 1/U_ii.
struct BandLU {
  int n = 0, lower = 0, upper = 0;
  std::vector<double> lmul, u, uinv;
};

struct FftPlan {
  int n = 0;
  int nstages = 0;
  int radix[kMaxStages] = {0};
  int ns[kMaxStages] = {0};
  std::vector<double> tw;  // tw[2t], tw[2t+1] = cos, sin of -2 pi t / n
};

struct HostTables {
  lmvd_config cfg{};
  std::vector<double> breakpoints;
  int n2 = 0, p = 0, nl = 0, nn = 0, hx = 0;
  std::vector<double> t, ts;         // knots of B (order p) and B* (order p+1)
  std::vector<double> tau, tau_s;    // Greville points
  RowTable E[3];                     // d^d B_j (tau_i)
  RowTable F0;                       // B*_j (tau_i)
  RowTable G[2];                     // d^d B_j (tau*_i)
  RowTable Es[3];                    // d^d B*_j (tau*_i)
  std::vector<double> dstar;         // (D* c)_j = dstar[j] (c_{j+1} - c_j)
  BandLU proj[3];                    // interpolation, Dirichlet rows, Neumann rows
  int a_lower = 0, a_upper = 0;      // band of A(k) = E*_2 - k^2 E*_0 with Robin rows
  std::vector<double> k1, k3;        // k1[l], k3[n_idx]
  FftPlan fz, fx;                    // complex FFTs of size m3 and m1/2
  std::vector<double> xtw;           // cos, sin of -2 pi k / m1, k < m1/2
  // rows i' of E_0 whose band starts at row i (lo(i') = i): emit_first[i], emit_cnt[i]
  std::vector<int32_t> emit_first, emit_cnt;
  // interior tau* rows i' (1..n2-1) of G_1 whose band starts at B row j: g1e_first[j], g1e_cnt[j]
  std::vector<int32_t> g1e_first, g1e_cnt;
  // tau rows i' whose last B* column (F_0 and F_1 = E_0 D* rows) is c row j: asc_first[j], asc_cnt[j]
  // (j = 0..n2); asc_w[(d n2 + i') kMaxW + q] multiplies c_{last(i') - q}, d = 0 (F_0), 1 (F_1)
  std::vector<int32_t> asc_first, asc_cnt;
  std::vector<double> asc_w;
  // bottom-up elimination of A(k) (rows n2 .. 0): per row i the number of
  // multipliers (rows i+1 .. i+nm) and of entries left of the diagonal
  // (columns i-1 .. i-ns) that can be nonzero (structure of A, union over
  // sampled k), and the offset of the row's nm + ns + 1 factor slots
  std::vector<int32_t> fac_nm, fac_ns, fac_off;
  int fac_slots = 0;
  // Values at the wall rows of the Neumann projection of interior values:
  // (E_0 P_N v)_0 = sum_{i=1}^{wall_k0} wall_w[i] v_i and
  // (E_0 P_N v)_{n2-1} = sum_{i=1}^{wall_k1} wall_w[wall_k0 + 1 + i] v_{n2-1-i}
  // (rows i = 0 and n2-1 of v do not enter P_N); the sums stop where the
  // remaining weights add up to at most 2^-60 of all of them.
  std::vector<double> wall_w;
  int wall_k0 = 0, wall_k1 = 0;
};

// Build all host tables.  Returns LMVD_OK or an error with `msg` set.
lmvd_status build_host_tables(const lmvd_config& cfg, HostTables& out, std::string& msg);

// Result of the pivot check of the A(k) elimination over every distinct k of a grid.
struct FactorCheck {
  double max_growth = 0.0;       // largest entry of an eliminated row over the row's largest entry in A
  double min_pivot_ratio = 0.0;  // smallest pivot over the row's largest entry in A
  int64_t bad_rows = 0;          // rows with a pivot below 1e-12 of the row or growth above the limit
  int64_t distinct_k = 0;        // nonzero k^2 checked
};
lmvd_status factor_check_host(const HostTables& H, double growth_max, FactorCheck& out);

// Values of the B (star = 0) or B* (star = 1) basis at arbitrary points of [-L2/2, L2/2], dense
// [points][n2 (+1)].
lmvd_status basis_values(const HostTables& H, int star, const std::vector<double>& y, std::vector<double>& out);

// Dense copy of a row table (row-major rows x cols).
std::vector<double> dense(const RowTable& r);

}  // namespace lmvd
