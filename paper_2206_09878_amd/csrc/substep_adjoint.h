// Adjoint of one substep (reverse mode of Algorithm time_advanceDNS in the reading of the forward path):
// the forward's intermediates are recomputed from the substep's inputs with the plan's linear operators
// (evaluation, transforms, projections, m^d, m^c) and elementwise kernels for the pointwise products,
// then every step is transposed in reverse order.  Transposes are taken in the real inner products
// <a, b> = sum Re(conj(a) b) over the stored entries of an S-field and sum f g over a physical field.
//
// Included once by lmvd.hip after its operators; uses its internal types.

namespace lmvd {

// ---------------------------------------------------------------------------
// elementwise kernels

enum AdjMult { AM_ONE = 0, AM_IK1 = 1, AM_IK3 = 2, AM_NIK1 = 3, AM_NIK3 = 4, AM_KSQ = 5 };

// y = (acc ? y : 0) + coef * mult(l, n) * x over `rows` rows of an S-field; with mask the (0,0) column gets 0
// added.  x may be NULL (then y is only cleared or kept).
__global__ void __launch_bounds__(kThreads) k_adj_axpy(DevPlan P, int rows, int mult, double coef, int mask,
                                                       const double2* __restrict__ x, double2* __restrict__ y,
                                                       int acc) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= ncol * rows) return;
  const size_t col = e % ncol;
  double2 v = zero2();
  if (x && !(mask && col == 0)) {
    const int l = int(col % size_t(P.nl)), ni = int(col / size_t(P.nl));
    const double k1 = P.k1[l], k3 = P.k3[ni];
    const double2 a = x[e];
    switch (mult) {
      case AM_IK1: v = make_double2(-k1 * a.y, k1 * a.x); break;
      case AM_IK3: v = make_double2(-k3 * a.y, k3 * a.x); break;
      case AM_NIK1: v = make_double2(k1 * a.y, -k1 * a.x); break;
      case AM_NIK3: v = make_double2(k3 * a.y, -k3 * a.x); break;
      case AM_KSQ: v = cscale(a, k1 * k1 + k3 * k3); break;
      default: v = a;
    }
    v = cscale(v, coef);
  }
  y[e] = acc ? cadd(y[e], v) : v;
}

// the Hermitian part of the l = 0 column, (f_{0,n} + conj f_{0,-n}) / 2 on both entries (the (0,0) entry
// keeps its real part), and with zero00 the (0,0) entry set to zero: the representative of a gradient on
// the S-fields the library accepts
__global__ void __launch_bounds__(kThreads) k_adj_herm(DevPlan P, int rows, double2* __restrict__ y, int zero00) {
  const int nn = P.nn, half = (nn + 1) / 2;
  const size_t ncol = size_t(nn) * P.nl;
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= size_t(rows) * half) return;
  const int j = int(t / half), ni = int(t % half);
  double2* row = y + size_t(j) * ncol;
  if (ni == 0) {
    const double2 a = row[0];
    row[0] = zero00 ? zero2() : make_double2(a.x, 0.0);
    return;
  }
  const size_t cp = size_t(ni) * P.nl, cm = size_t(nn - ni) * P.nl;
  const double2 a = row[cp], b = row[cm];
  const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  row[cp] = h;
  row[cm] = make_double2(h.x, -h.y);
}

// (0,0) column <-> real vector of n2 rows: mode 0 writes the S-field column from v (imaginary part 0);
// mode 1 adds the real part of the column to v
__global__ void k_adj_meancol(DevPlan P, int mode, double2* __restrict__ f, double* __restrict__ v) {
  const size_t ncol = size_t(P.nn) * P.nl;
  const int j = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= P.n2) return;
  if (mode == 0) f[size_t(j) * ncol] = make_double2(v[j], 0.0);
  else v[j] += f[size_t(j) * ncol].x;
}

// x = 0 on n doubles (a fill kernel, so that the adjoint stays free of memset nodes when captured)
__global__ void __launch_bounds__(kThreads) k_adj_zero(double* __restrict__ x, size_t n) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// v = (acc ? v : 0) + a x (+ b y) on real vectors of n
__global__ void k_adj_vaxpy(int n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                            double* __restrict__ v, int acc) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = acc ? v[i] : 0.0;
  if (x) s += a * x[i];
  if (y) s += b * y[i];
  v[i] = s;
}

// pointwise products of the forward recomputation and their transposes on the physical grid (n points)
enum AdjPoint {
  AP_RZ = 0,      // out = (-(m.grad z) + rhoD lap) / rho
  AP_RHOT = 1,    // out = f'(z) zt
  AP_L = 2,       // out = -(grad z . mc) / rho
  AP_RZ_T = 3,    // from R_bar: m_bar_i = -R_bar z_i / rho; z_i_bar, lap_bar, zp_bar accumulated
  AP_RHOT_T = 4,  // from r_bar: zt_bar = f' r_bar; zp_bar += f'' zt r_bar
  AP_L_T = 5,     // from L_bar: mc_bar_i = -L_bar z_i / rho; z_i_bar, zp_bar accumulated
  AP_FLUX_T = 6   // from T_bar (6 pairs), u_bar (3), rho_bar (gravity): m_bar_i; zp_bar accumulated
};

struct AdjPointArgs {
  const double* zp;        // z on the grid
  const double* g[3];      // d z / d x_i
  const double* lap;       // lap z
  const double* m[3];      // m^d (R_z), m^c (L), m (fluxes) on the grid
  const double* zt;        // z_t on the grid (rho_t)
  const double* in[10];    // cotangents: R_bar / r_bar / L_bar in in[0]; fluxes: T_bar pairs 0..5, u_bar 6..8,
                           // rho_bar 9
  double* out[3];          // forward output in out[0]; transposes: m_bar_i (or zt_bar in out[0])
  double* zpb;             // accumulated adjoints of z, grad z and lap z on the grid
  double* gb[3];
  double* lapb;
};

__global__ void __launch_bounds__(kThreads) k_adj_point(DevPlan P, int mode, size_t n, AdjPointArgs A) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double z = A.zp[i];
  const double den = P.rho_h - P.drho * z;  // rho = rho_l rho_h / den
  const double rinv = den * P.inv_rlrh;     // 1 / rho, linear in z
  const double drinv = -P.drho * P.inv_rlrh;  // d(1/rho)/dz
  const double rho = 1.0 / rinv;
  const double fp = rho * rho * P.drho * P.inv_rlrh;  // f'(z)
  switch (mode) {
    case AP_RZ: {
      const double a = -(A.m[0][i] * A.g[0][i] + A.m[1][i] * A.g[1][i] + A.m[2][i] * A.g[2][i]) + P.rhoD * A.lap[i];
      A.out[0][i] = a * rinv;
      break;
    }
    case AP_RHOT: A.out[0][i] = fp * A.zt[i]; break;
    case AP_L: {
      const double a = A.g[0][i] * A.m[0][i] + A.g[1][i] * A.m[1][i] + A.g[2][i] * A.m[2][i];
      A.out[0][i] = -a * rinv;
      break;
    }
    case AP_RZ_T: {
      const double rb = A.in[0][i];
      const double a = -(A.m[0][i] * A.g[0][i] + A.m[1][i] * A.g[1][i] + A.m[2][i] * A.g[2][i]) + P.rhoD * A.lap[i];
      for (int k = 0; k < 3; ++k) {
        A.out[k][i] = -rb * rinv * A.g[k][i];
        A.gb[k][i] += -rb * rinv * A.m[k][i];
      }
      A.lapb[i] += rb * rinv * P.rhoD;
      A.zpb[i] += rb * drinv * a;
      break;
    }
    case AP_RHOT_T: {
      const double rb = A.in[0][i];
      const double fpp = 2.0 * fp * P.drho * rho * P.inv_rlrh;  // f''(z) = 2 (rho_h - rho_l) f' rho / (rho_l rho_h)
      A.out[0][i] = fp * rb;
      A.zpb[i] += fpp * A.zt[i] * rb;
      break;
    }
    case AP_L_T: {
      const double lb = A.in[0][i];
      const double a = A.g[0][i] * A.m[0][i] + A.g[1][i] * A.m[1][i] + A.g[2][i] * A.m[2][i];
      for (int k = 0; k < 3; ++k) {
        A.out[k][i] = -lb * rinv * A.g[k][i];
        A.gb[k][i] += -lb * rinv * A.m[k][i];
      }
      A.zpb[i] += -lb * drinv * a;
      break;
    }
    case AP_FLUX_T: {
      // T_ab = -m_a m_b / rho for the pairs (00, 01, 02, 11, 12, 22); u_a = m_a / rho
      const double m0 = A.m[0][i], m1 = A.m[1][i], m2 = A.m[2][i];
      const double t00 = A.in[0][i], t01 = A.in[1][i], t02 = A.in[2][i], t11 = A.in[3][i], t12 = A.in[4][i],
                   t22 = A.in[5][i];
      const double u0 = A.in[6][i], u1 = A.in[7][i], u2 = A.in[8][i];
      A.out[0][i] = -rinv * (2.0 * t00 * m0 + t01 * m1 + t02 * m2) + u0 * rinv;
      A.out[1][i] = -rinv * (t01 * m0 + 2.0 * t11 * m1 + t12 * m2) + u1 * rinv;
      A.out[2][i] = -rinv * (t02 * m0 + t12 * m1 + 2.0 * t22 * m2) + u2 * rinv;
      const double q = t00 * m0 * m0 + t01 * m0 * m1 + t02 * m0 * m2 + t11 * m1 * m1 + t12 * m1 * m2 + t22 * m2 * m2;
      // d/drho of -m_a m_b / rho is m_a m_b / rho^2; of m_a / rho is -m_a / rho^2
      const double rhob = A.in[9][i] + rinv * rinv * (q - (u0 * m0 + u1 * m1 + u2 * m2));
      A.zpb[i] += rhob * fp;
      break;
    }
    default: break;
  }
}

// ---------------------------------------------------------------------------
// workspace of the adjoint: the substep's workspace, then these fields
struct AdjLayout {
  size_t S = 0, Ss = 0, Ph = 0;  // bytes of an S-field (B), a B* S-field, a physical field
  int kf = 0;
  // physical fields
  size_t zp, g[3], lap, mdp[3], ztp, mcp, mp[3], zpb, gb[3], lapb, pt[10];
  // S-fields (B) and B* fields
  size_t md1, md3, md2, rz, ztc, ztn, rhot, mc1, mc3, mc2, m1, m3, m2;
  size_t ztb, rzb, t1, t2, t3, t4, nb[3], dnb[3], tb[6], ub[3], zb, mcb1, mcb3, mcb2, mdb1, mdb3, mdb2;
  size_t vec;  // 4 real vectors of n2
  size_t bytes = 0;
};

static AdjLayout adjoint_layout(const lmvd_plan_s* p, int kf) {
  const HostTables& H = p->H;
  AdjLayout L;
  L.kf = kf;
  const size_t ncol = size_t(H.nn) * H.nl;
  L.S = ncol * H.n2 * 16;
  L.Ss = ncol * (H.n2 + 1) * 16;
  L.Ph = size_t(H.n2) * H.cfg.m3 * H.cfg.m1 * 8;
  size_t o = align256(p->ws.bytes);
  auto take = [&](size_t b) { size_t r = o; o = align256(o + b); return r; };
  L.zp = take(L.Ph);
  for (auto& x : L.g) x = take(L.Ph);
  L.lap = take(L.Ph);
  for (auto& x : L.mdp) x = take(L.Ph);
  L.ztp = take(L.Ph * size_t(kf + 1));
  L.mcp = take(L.Ph * 3 * size_t(std::max(kf, 1)));
  for (auto& x : L.mp) x = take(L.Ph);
  L.zpb = take(L.Ph);
  for (auto& x : L.gb) x = take(L.Ph);
  L.lapb = take(L.Ph);
  for (auto& x : L.pt) x = take(L.Ph);
  for (size_t* x : {&L.md1, &L.md3, &L.rz, &L.ztc, &L.ztn, &L.rhot, &L.mc1, &L.mc3, &L.m1, &L.m3, &L.ztb, &L.rzb,
                    &L.zb, &L.mcb1, &L.mcb3, &L.mdb1, &L.mdb3})
    *x = take(L.S);
  // scratch fields hold B* coefficients too (F0^T writes n2 + 1 rows)
  for (size_t* x : {&L.t1, &L.t2, &L.t3, &L.t4}) *x = take(L.Ss);
  for (auto& x : L.nb) x = take(L.S);
  for (auto& x : L.dnb) x = take(L.S);
  for (auto& x : L.tb) x = take(L.S);
  for (auto& x : L.ub) x = take(L.S);
  for (size_t* x : {&L.md2, &L.mc2, &L.m2, &L.mcb2, &L.mdb2}) *x = take(L.Ss);
  L.vec = take(size_t(4) * H.n2 * 8);
  L.bytes = o;
  return L;
}

// ---------------------------------------------------------------------------
// the adjoint substep

struct AdjCtx {
  Ctx c;
  AdjLayout L;
  size_t ncol, nS, nSs, nPh;
  dim3 gS, gSs, gPh, gC;
  template <typename T>
  T* at(size_t off) const {
    return c.at<T>(off);
  }
  double2* S(size_t off) const { return at<double2>(off); }
  double* Ph(size_t off) const { return at<double>(off); }
};

static AdjCtx adj_ctx(lmvd_plan_s* p, char* ws, hipStream_t s, int kf) {
  AdjCtx a{Ctx{p, ws, s}, adjoint_layout(p, kf), 0, 0, 0, 0, {}, {}, {}, {}};
  a.ncol = ncols(p);
  a.nS = a.ncol * p->H.n2;
  a.nSs = a.ncol * (p->H.n2 + 1);
  a.nPh = size_t(p->H.n2) * p->H.cfg.m3 * p->H.cfg.m1;
  a.gS = dim3(unsigned((a.nS + kThreads - 1) / kThreads));
  a.gSs = dim3(unsigned((a.nSs + kThreads - 1) / kThreads));
  a.gPh = dim3(unsigned((a.nPh + kThreads - 1) / kThreads));
  a.gC = dim3(unsigned((a.ncol + kThreads - 1) / kThreads));
  return a;
}

// y (+)= coef mult x over an S-field (star: n2 + 1 rows)
static void axpy(const AdjCtx& a, const double2* x, double2* y, double coef = 1.0, int mult = AM_ONE, bool acc = true,
                 bool star = false, bool mask = false) {
  hipLaunchKernelGGL(k_adj_axpy, star ? a.gSs : a.gS, dim3(kThreads), 0, a.c.s, a.c.p->D,
                     star ? a.c.p->H.n2 + 1 : a.c.p->H.n2, mult, coef, mask ? 1 : 0, x, y, acc ? 1 : 0);
}
static void clear(const AdjCtx& a, double2* y, bool star = false) { axpy(a, nullptr, y, 0.0, AM_ONE, false, star); }

// coefficients -> physical field: Inv(mult E_kind coeffs)
static lmvd_status to_phys(const AdjCtx& a, const void* coeffs, int kind, double* phys, int mult = MU_ONE) {
  return plane_phase<PH_TOPHYS>(a.c, {ev(coeffs, kind, mult)}, {}, phys, nullptr);
}
// physical field -> values at tau (forward transform)
static lmvd_status to_vals(const AdjCtx& a, const double* phys, double2* vals) {
  return plane_phase<PH_FROMPHYS>(a.c, {}, {vals}, nullptr, phys);
}
// transpose of the inverse transform: physical cotangent -> values cotangent
static lmvd_status inv_t(const AdjCtx& a, const double* phys, double2* vals) {
  lmvd_status st = to_vals(a, phys, vals);
  if (st != LMVD_OK) return st;
  hipLaunchKernelGGL(k_scale_modes, a.gS, dim3(kThreads), 0, a.c.s, a.c.p->D, vals, vals, 0);
  return LMVD_OK;
}
// transpose of the forward transform: values cotangent -> physical cotangent (vals is overwritten)
static lmvd_status fwd_t(const AdjCtx& a, double2* vals, double* phys) {
  hipLaunchKernelGGL(k_scale_modes, a.gS, dim3(kThreads), 0, a.c.s, a.c.p->D, vals, vals, 1);
  return plane_phase<PH_TOPHYS>(a.c, {ev(vals, EV_IDENT)}, {}, phys, nullptr);
}
static void eval_t(const AdjCtx& a, int kind, const double2* vals, double2* coeffs) {
  const dim3 g(a.gC.x, unsigned(kind == EV_F0 ? a.c.p->H.n2 + 1 : a.c.p->H.n2));
  hipLaunchKernelGGL(k_evaluate_t, g, dim3(kThreads), 0, a.c.s, a.c.p->D, kind, vals, coeffs);
}
// R A^{-T} of `kind` for n independent (coeffs, vals) pairs in one launch; a pair may be in place
static void proj_t_n(const AdjCtx& a, int kind, int n, const double2* const* coeffs, double2* const* vals) {
  ProjTJobs J{};
  for (int j = 0; j < n; ++j) J.in[j] = coeffs[j], J.out[j] = vals[j];
  hipLaunchKernelGGL(k_project_t, dim3(a.gC.x, unsigned(n)), dim3(kThreads), 0, a.c.s, a.c.p->D, kind, J);
}
static void proj_t(const AdjCtx& a, int kind, const double2* coeffs, double2* vals) {
  proj_t_n(a, kind, 1, &coeffs, &vals);
}
// coeffs_bar (+)= E_kind^T Inv^T(phys_bar), through the two scratch fields t, u
static lmvd_status phys_to_coef_t(const AdjCtx& a, const double* physb, int kind, double2* coefb, double2* t,
                                  double2* u, bool acc, int mult = AM_ONE) {
  lmvd_status st = inv_t(a, physb, t);
  if (st != LMVD_OK) return st;
  if (mult != AM_ONE) axpy(a, t, t, 1.0, mult, false);
  const bool star = (kind == EV_F0);
  if (!acc) {
    eval_t(a, kind, t, coefb);
    return LMVD_OK;
  }
  eval_t(a, kind, t, u);
  axpy(a, u, coefb, 1.0, AM_ONE, true, star);
  return LMVD_OK;
}
static void mc_t(const AdjCtx& a, const double2* m1b, const double2* m2b, const double2* m3b, double2* rhotb) {
  double2* scr = a.c.at<double2>(a.c.p->ws.off_yt);
  hipLaunchKernelGGL(k_mc_t, a.gC, dim3(kThreads), 0, a.c.s, a.c.p->D, m1b, m2b, m3b, rhotb, scr);
}

static lmvd_status run_substep_adjoint(lmvd_plan_s* p, const lmvd_substep_args* fa, const lmvd_substep_grads* g,
                                       char* ws, hipStream_t s, int kf) {
  const HostTables& H = p->H;
  const AdjCtx a = adj_ctx(p, ws, s, kf);
  const AdjLayout& L = a.L;
  const double dt = H.cfg.dt;
  const int n2 = H.n2;
  lmvd_status st = LMVD_OK;
#define ADJ_OK(x)             \
  do {                        \
    st = (x);                 \
    if (st != LMVD_OK) return st; \
  } while (0)
  auto cS = [](const void* q) { return static_cast<const double2*>(q); };
  const double2* z = cS(fa->z);
  double* zp = a.Ph(L.zp);
  double* gz[3] = {a.Ph(L.g[0]), a.Ph(L.g[1]), a.Ph(L.g[2])};
  double* lap = a.Ph(L.lap);
  double* mdp[3] = {a.Ph(L.mdp[0]), a.Ph(L.mdp[1]), a.Ph(L.mdp[2])};
  double* mp[3] = {a.Ph(L.mp[0]), a.Ph(L.mp[1]), a.Ph(L.mp[2])};
  double* pt[10];
  for (int i = 0; i < 10; ++i) pt[i] = a.Ph(L.pt[i]);
  auto ztp = [&](int k) { return a.Ph(L.ztp + size_t(k) * L.Ph); };
  auto mcp = [&](int k, int i) { return a.Ph(L.mcp + (size_t(k) * 3 + i) * L.Ph); };
  double2 *md1 = a.S(L.md1), *md2 = a.S(L.md2), *md3 = a.S(L.md3);
  double2 *rz = a.S(L.rz), *ztc = a.S(L.ztc), *ztn = a.S(L.ztn), *rhot = a.S(L.rhot);
  double2 *mc1 = a.S(L.mc1), *mc2 = a.S(L.mc2), *mc3 = a.S(L.mc3);
  double2 *t1 = a.S(L.t1), *t2 = a.S(L.t2), *t3 = a.S(L.t3), *t4 = a.S(L.t4);
  auto pointwise = [&](int mode, AdjPointArgs A) {
    hipLaunchKernelGGL(k_adj_point, a.gPh, dim3(kThreads), 0, s, p->D, mode, a.nPh, A);
  };

  // ---- forward recomputation ----
  // m^d coefficients (eqs. phi_poisson, md_recon): the substep's own m^d job with the plan's factors, its
  // values at tau written to scratch, where the substep runs it; else the solve with the LU formed per call
  if (H.p == 8) {
    const int nth = 2 * H.nl * ((H.nn + 1) / 2);
    const MdArgs margs{cS(fa->phi2), cS(fa->omega2), fa->m1bar, fa->m3bar, a.c.at<double2>(p->ws.off_yt),
                       t2, t3, t4, md2, md1, md3};
    const dim3 gm((unsigned(nth) + kThreads - 1) / kThreads, 1);  // job 0 only
    if (p->fac_la == 7)
      col<JobPrologue<7, 7, 8>>(a.c, gm, 0, {1, margs, ValuesZArgs{}, GuessArgs{}});
    else
      col<JobPrologue<8, 8, 8>>(a.c, gm, 0, {1, margs, ValuesZArgs{}, GuessArgs{}});
  } else {
    solveA<0>(a.c, cS(fa->phi2), cS(fa->omega2), fa->m1bar, fa->m3bar, md2, md1, md3);
  }
  // z and its derivatives on the grid
  ADJ_OK(to_phys(a, z, EV_E0, zp));
  ADJ_OK(to_phys(a, z, EV_E0, gz[0], MU_IK1));
  ADJ_OK(to_phys(a, z, EV_E1, gz[1]));
  ADJ_OK(to_phys(a, z, EV_E0, gz[2], MU_IK3));
  ADJ_OK(to_phys(a, z, EV_LAP, lap));
  ADJ_OK(to_phys(a, md1, EV_E0, mdp[0]));
  ADJ_OK(to_phys(a, md2, EV_F0, mdp[1]));
  ADJ_OK(to_phys(a, md3, EV_E0, mdp[2]));
  // R_z = P_N^{-1} Fwd((-(m^d . grad z) + rhoD lap z) / rho)
  {
    AdjPointArgs A{};
    A.zp = zp;
    for (int i = 0; i < 3; ++i) A.g[i] = gz[i], A.m[i] = mdp[i];
    A.lap = lap;
    A.out[0] = pt[0];
    pointwise(AP_RZ, A);
    ADJ_OK(to_vals(a, pt[0], t1));
    proj(a.c, 2, t1, rz);
  }
  // guess (eq. dzdt_guesses) or zero
  double co[4];
  if (fa->stage == 0) {
    co[0] = 2.0; co[1] = -2.0 - 0.5 * H.cfg.beta_n; co[2] = H.cfg.beta_n; co[3] = -0.5 * H.cfg.beta_n;
  } else {
    co[0] = 4.0 + H.cfg.beta_p; co[1] = -5.0 - 2.0 * H.cfg.beta_p; co[2] = H.cfg.beta_p; co[3] = 1.0;
  }
  const bool zero_guess = fa->guess_mode == 1;
  if (zero_guess) {
    clear(a, ztc);
  } else {
    axpy(a, z, ztc, co[0] / dt, AM_ONE, false);
    for (int h = 0; h < 3; ++h) axpy(a, cS(fa->z_hist[h]), ztc, co[h + 1] / dt);
  }
  // fixed-point iterations; the grid values of every iterate's z_t and m^c are kept
  // rho_t values at tau (in t1) of an iterate, its z_t kept on the grid
  auto rhot_vals = [&](const double2* zt, double* ztphys) -> lmvd_status {
    lmvd_status r = to_phys(a, zt, EV_E0, ztphys);
    if (r != LMVD_OK) return r;
    AdjPointArgs A{};
    A.zp = zp;
    A.zt = ztphys;
    A.out[0] = pt[0];
    pointwise(AP_RHOT, A);
    return to_vals(a, pt[0], t1);
  };
  for (int k = 0; k < kf; ++k) {
    // m^c values at tau by the substep's fused kernel (mc1, mc2, mc3 hold values here), then on the grid
    ADJ_OK(rhot_vals(ztc, ztp(k)));
    launch_mc(a.c, t1, nullptr, nullptr, nullptr, mc1, mc2, mc3, nullptr, nullptr, nullptr);
    ADJ_OK(to_phys(a, mc1, EV_IDENT, mcp(k, 0)));
    ADJ_OK(to_phys(a, mc2, EV_IDENT, mcp(k, 1)));
    ADJ_OK(to_phys(a, mc3, EV_IDENT, mcp(k, 2)));
    AdjPointArgs A{};
    A.zp = zp;
    for (int i = 0; i < 3; ++i) A.g[i] = gz[i], A.m[i] = mcp(k, i);
    A.out[0] = pt[0];
    pointwise(AP_L, A);
    ADJ_OK(to_vals(a, pt[0], t1));
    proj(a.c, 2, t1, ztn);
    axpy(a, rz, ztn);
    std::swap(ztc, ztn);
  }
  // final m^c coefficients (eqs. COM_fourier, CF_fourier, mc_recon, mc_mean) by the substep's fused kernel in
  // its final-iterate form (rho_t coefficients, c and m_par; its values at tau go to scratch), then
  // m1 = (k1/k) m_par, m3 = (k3/k) m_par; and m = m^d + m^c on the grid
  ADJ_OK(rhot_vals(ztc, ztp(kf)));
  {
    double2* mpar = a.c.at<double2>(p->ws.off_mpar);
    launch_mc(a.c, t1, nullptr, nullptr, nullptr, t2, t3, t4, rhot, mc2, mpar);
    hipLaunchKernelGGL(k_mc13, a.gS, dim3(kThreads), 0, s, p->D, mpar, mc1, mc3);
  }
  double2 *m1 = a.S(L.m1), *m2 = a.S(L.m2), *m3 = a.S(L.m3);
  axpy(a, md1, m1, 1.0, AM_ONE, false);
  axpy(a, mc1, m1);
  axpy(a, md2, m2, 1.0, AM_ONE, false, true);
  axpy(a, mc2, m2, 1.0, AM_ONE, true, true);
  axpy(a, md3, m3, 1.0, AM_ONE, false);
  axpy(a, mc3, m3);
  ADJ_OK(to_phys(a, m1, EV_E0, mp[0]));
  ADJ_OK(to_phys(a, m2, EV_F0, mp[1]));
  ADJ_OK(to_phys(a, m3, EV_E0, mp[2]));

  // ---- reverse sweep ----
  // cotangents of the outputs (Hermitian parts: the library's S-fields have a Hermitian l = 0 column)
  double2 *ztb = a.S(L.ztb), *rzb = a.S(L.rzb), *zb = a.S(L.zb);
  double2 *rphb = t3, *romb = t4;  // cotangents of RHS_phi2, RHS_Omega2
  double* vec = a.at<double>(L.vec);
  double *rm1b = vec, *rm3b = vec + n2, *tmpv = vec + 2 * n2;
  const double wout = (fa->stage == 0) ? 0.5 * dt : dt;  // d out / d RHS of this stage
  auto herm = [&](double2* f, bool star, bool zero00) {
    const int rows = star ? n2 + 1 : n2;
    const size_t nt = size_t(rows) * ((H.nn + 1) / 2);
    hipLaunchKernelGGL(k_adj_herm, dim3(unsigned((nt + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, p->D, rows,
                       f, zero00 ? 1 : 0);
  };
  auto vaxpy = [&](double av, const double* x, double bv, const double* y, double* v, bool acc) {
    hipLaunchKernelGGL(k_adj_vaxpy, dim3(unsigned((n2 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n2, av, x,
                       bv, y, v, acc ? 1 : 0);
  };
  // RK2: out = X + wout R (- dt/2 R_prev at stage '); z_out = z + wout zt (- dt/2 zt_prev)
  axpy(a, cS(g->rhs_phi2), rphb, 1.0, AM_ONE, false);
  axpy(a, cS(g->phi2_out), rphb, wout);
  axpy(a, cS(g->rhs_omega2), romb, 1.0, AM_ONE, false);
  axpy(a, cS(g->omega2_out), romb, wout);
  herm(rphb, false, true);
  herm(romb, false, true);
  vaxpy(1.0, g->rhs_m1, wout, g->m1bar_out, rm1b, false);
  vaxpy(1.0, g->rhs_m3, wout, g->m3bar_out, rm3b, false);
  axpy(a, cS(g->zt), ztb, 1.0, AM_ONE, false);
  axpy(a, cS(g->z_out), ztb, wout);
  herm(ztb, false, false);
  // z_bar starts from the direct path z -> z_out
  axpy(a, cS(g->z_out), zb, 1.0, AM_ONE, false);
  if (fa->stage == 1) {
    if (g->rhs_phi2_prev) axpy(a, cS(g->phi2_out), static_cast<double2*>(g->rhs_phi2_prev), -0.5 * dt, AM_ONE, false);
    if (g->rhs_omega2_prev)
      axpy(a, cS(g->omega2_out), static_cast<double2*>(g->rhs_omega2_prev), -0.5 * dt, AM_ONE, false);
    if (g->zt_prev) axpy(a, cS(g->z_out), static_cast<double2*>(g->zt_prev), -0.5 * dt, AM_ONE, false);
    if (g->rhs_m1_prev) vaxpy(-0.5 * dt, g->m1bar_out, 0.0, nullptr, g->rhs_m1_prev, false);
    if (g->rhs_m3_prev) vaxpy(-0.5 * dt, g->m3bar_out, 0.0, nullptr, g->rhs_m3_prev, false);
  }

  // RHS (steps 4 and 5): R_phi = P_D^{-1} mask(-k^2 N2 - d/dy(i k1 N1 + i k3 N3) + k^2 g rho),
  // R_Omega = P_D^{-1} mask(i k3 N1 - i k1 N3), R<m>1,3 = P_N^{-1} E1 <T12>, E1 <T32>
  double2* nb[3] = {a.S(L.nb[0]), a.S(L.nb[1]), a.S(L.nb[2])};
  double2* dnb[3] = {a.S(L.dnb[0]), a.S(L.dnb[1]), a.S(L.dnb[2])};
  double2* tb[6];
  for (int i = 0; i < 6; ++i) tb[i] = a.S(L.tb[i]);
  double2* ub[3] = {a.S(L.ub[0]), a.S(L.ub[1]), a.S(L.ub[2])};
  {  // v_bar of R_phi into t1, of R_Omega into t2
    const double2* in[2] = {rphb, romb};
    double2* out[2] = {t1, t2};
    proj_t_n(a, 1, 2, in, out);
  }
  axpy(a, t1, nb[1], -1.0, AM_KSQ, false, false, true);
  axpy(a, t1, dnb[0], 1.0, AM_IK1, false, false, true);
  axpy(a, t1, dnb[2], 1.0, AM_IK3, false, false, true);
  axpy(a, t2, nb[0], 1.0, AM_NIK3, false, false, true);
  axpy(a, t2, nb[2], 1.0, AM_IK1, false, false, true);
  // gravity: rho values cotangent = k^2 g v_bar (masked), on the grid through Fwd^T
  axpy(a, t1, rhot, H.cfg.g, AM_KSQ, false, false, true);
  ADJ_OK(fwd_t(a, rhot, pt[9]));
  // N_i = i k1 E0 T_i1 + E1 T_i2 + i k3 E0 T_i3, dN_i likewise with E1, E2: T_bar of the stored pairs
  const int pair[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  for (int q = 0; q < 6; ++q) clear(a, tb[q]);
  for (int i = 0; i < 3; ++i) {
    const bool has_dn = (i != 1);  // dN_2 does not enter (its d/dy is taken of N_1 and N_3 only)
    // j = 0: E0^T(-i k1 N_bar) + E1^T(-i k1 dN_bar)
    axpy(a, nb[i], t1, 1.0, AM_NIK1, false);
    eval_t(a, EV_E0, t1, t2);
    axpy(a, t2, tb[pair[i][0]]);
    if (has_dn) {
      axpy(a, dnb[i], t1, 1.0, AM_NIK1, false);
      eval_t(a, EV_E1, t1, t2);
      axpy(a, t2, tb[pair[i][0]]);
    }
    // j = 1: E1^T N_bar + E2^T dN_bar
    eval_t(a, EV_E1, nb[i], t2);
    axpy(a, t2, tb[pair[i][1]]);
    if (has_dn) {
      eval_t(a, EV_E2, dnb[i], t2);
      axpy(a, t2, tb[pair[i][1]]);
    }
    // j = 2: E0^T(-i k3 N_bar) + E1^T(-i k3 dN_bar)
    axpy(a, nb[i], t1, 1.0, AM_NIK3, false);
    eval_t(a, EV_E0, t1, t2);
    axpy(a, t2, tb[pair[i][2]]);
    if (has_dn) {
      axpy(a, dnb[i], t1, 1.0, AM_NIK3, false);
      eval_t(a, EV_E1, t1, t2);
      axpy(a, t2, tb[pair[i][2]]);
    }
  }
  // plane means: <T12>_bar (pair 1) and <T32>_bar (pair 4) += E1^T P_N^T R<m>_bar (real parts)
  for (int q = 0; q < 2; ++q) {
    clear(a, t1);
    hipLaunchKernelGGL(k_adj_meancol, dim3(unsigned((n2 + 63) / 64)), dim3(64), 0, s, p->D, 0, t1,
                       q == 0 ? rm1b : rm3b);
    proj_t(a, 2, t1, t2);
    eval_t(a, EV_E1, t2, t1);
    vaxpy(0.0, nullptr, 0.0, nullptr, tmpv, false);
    hipLaunchKernelGGL(k_adj_meancol, dim3(unsigned((n2 + 63) / 64)), dim3(64), 0, s, p->D, 1, t1, tmpv);
    clear(a, t2);
    hipLaunchKernelGGL(k_adj_meancol, dim3(unsigned((n2 + 63) / 64)), dim3(64), 0, s, p->D, 0, t2, tmpv);
    axpy(a, t2, tb[q == 0 ? 1 : 4]);
  }
  // T_hat = P0^{-1} (values of T): V_ab = P0^T T_hat_bar, the six in place in one launch
  static_assert(kProjTJobs >= 6, "six stress components per launch");
  proj_t_n(a, 0, 6, tb, tb);
  // viscous part, formed spectrally from u_hat: s_ab = mu (D_b u_a + D_a u_b) - 2/3 mu delta_ab sum_c D_c u_c,
  // D_0 = i k1 E0, D_1 = E1, D_2 = i k3 E0
  const double mu = H.cfg.mu;
  for (int i = 0; i < 3; ++i) clear(a, ub[i]);
  auto add_Dt = [&](int c, const double2* v, double coef, double2* dst) {
    // dst += coef D_c^T v
    if (c == 1) {
      eval_t(a, EV_E1, v, t2);
    } else {
      axpy(a, v, t1, 1.0, c == 0 ? AM_NIK1 : AM_NIK3, false);
      eval_t(a, EV_E0, t1, t2);
    }
    axpy(a, t2, dst, coef);
  };
  for (int aa = 0; aa < 3; ++aa)
    for (int bb = aa; bb < 3; ++bb) {
      const double2* V = tb[pair[aa][bb]];
      if (aa == bb) {
        add_Dt(aa, V, 2.0 * mu, ub[aa]);
      } else {
        add_Dt(bb, V, mu, ub[aa]);
        add_Dt(aa, V, mu, ub[bb]);
      }
    }
  axpy(a, tb[0], t4, 1.0, AM_ONE, false);  // sum of the diagonal V_aa
  axpy(a, tb[3], t4);
  axpy(a, tb[5], t4);
  for (int c = 0; c < 3; ++c) add_Dt(c, t4, -2.0 / 3.0 * mu, ub[c]);
  // convective part on the grid: T_bar_ab = Fwd^T V_ab; u_bar = Fwd^T P0^T u_hat_bar
  for (int q = 0; q < 6; ++q) ADJ_OK(fwd_t(a, tb[q], pt[q]));
  proj_t_n(a, 0, 3, ub, ub);  // u_hat_bar -> P0^T u_hat_bar in place (ub is not read again)
  for (int i = 0; i < 3; ++i) ADJ_OK(fwd_t(a, ub[i], pt[6 + i]));
  double* zpb = a.Ph(L.zpb);
  double* gb[3] = {a.Ph(L.gb[0]), a.Ph(L.gb[1]), a.Ph(L.gb[2])};
  double* lapb = a.Ph(L.lapb);
  for (double* q : {zpb, gb[0], gb[1], gb[2], lapb})
    hipLaunchKernelGGL(k_adj_zero, a.gPh, dim3(kThreads), 0, s, q, a.nPh);
  // m on the grid is overwritten by its cotangent (each point reads m before it writes)
  double* mpb[3] = {mp[0], mp[1], mp[2]};
  {
    AdjPointArgs A{};
    A.zp = zp;
    for (int i = 0; i < 3; ++i) A.m[i] = mp[i], A.out[i] = mpb[i];
    for (int i = 0; i < 10; ++i) A.in[i] = pt[i];
    A.zpb = zpb;
    pointwise(AP_FLUX_T, A);
  }
  // m = m^d + m^c (m2 in B*): coefficient cotangents
  double2 *mcb1 = a.S(L.mcb1), *mcb2 = a.S(L.mcb2), *mcb3 = a.S(L.mcb3);
  ADJ_OK(phys_to_coef_t(a, mpb[0], EV_E0, mcb1, t1, t2, false));
  ADJ_OK(phys_to_coef_t(a, mpb[1], EV_F0, mcb2, t1, t2, false));
  ADJ_OK(phys_to_coef_t(a, mpb[2], EV_E0, mcb3, t1, t2, false));
  double2 *mdb1 = a.S(L.mdb1), *mdb2 = a.S(L.mdb2), *mdb3 = a.S(L.mdb3);
  axpy(a, mcb1, mdb1, 1.0, AM_ONE, false);
  axpy(a, mcb2, mdb2, 1.0, AM_ONE, false, true);
  axpy(a, mcb3, mdb3, 1.0, AM_ONE, false);
  // diagnostic outputs m^d, m^c of the substep
  if (g->md[0]) axpy(a, cS(g->md[0]), mdb1);
  if (g->md[1]) axpy(a, cS(g->md[1]), mdb2, 1.0, AM_ONE, true, true);
  if (g->md[2]) axpy(a, cS(g->md[2]), mdb3);
  if (g->mc[0]) axpy(a, cS(g->mc[0]), mcb1);
  if (g->mc[1]) axpy(a, cS(g->mc[1]), mcb2, 1.0, AM_ONE, true, true);
  if (g->mc[2]) axpy(a, cS(g->mc[2]), mcb3);

  // final m^c from z_t^{kf}: rho_t_bar = MC^T m^c_bar; r_bar = Fwd^T P0^T rho_t_bar; rho_t = f'(z) z_t
  auto rhot_t = [&](int k, double2* ztb_out, bool acc) -> lmvd_status {
    mc_t(a, mcb1, mcb2, mcb3, t1);
    proj_t(a, 0, t1, t2);
    lmvd_status r = fwd_t(a, t2, pt[0]);
    if (r != LMVD_OK) return r;
    AdjPointArgs A{};
    A.zp = zp;
    A.zt = ztp(k);
    A.in[0] = pt[0];
    A.out[0] = pt[1];
    A.zpb = zpb;
    pointwise(AP_RHOT_T, A);
    return phys_to_coef_t(a, pt[1], EV_E0, ztb_out, t1, t2, acc);
  };
  ADJ_OK(rhot_t(kf, ztb, true));
  // iterations in reverse: z_t^k = P_N^{-1} Fwd(L(z_t^{k-1})) + R_z
  clear(a, rzb);
  for (int k = kf - 1; k >= 0; --k) {
    axpy(a, ztb, rzb);
    proj_t(a, 2, ztb, t1);
    ADJ_OK(fwd_t(a, t1, pt[0]));
    AdjPointArgs A{};
    A.zp = zp;
    for (int i = 0; i < 3; ++i) A.g[i] = gz[i], A.m[i] = mcp(k, i), A.out[i] = pt[1 + i], A.gb[i] = gb[i];
    A.in[0] = pt[0];
    A.zpb = zpb;
    pointwise(AP_L_T, A);
    ADJ_OK(phys_to_coef_t(a, pt[1], EV_E0, mcb1, t1, t2, false));
    ADJ_OK(phys_to_coef_t(a, pt[2], EV_F0, mcb2, t1, t2, false));
    ADJ_OK(phys_to_coef_t(a, pt[3], EV_E0, mcb3, t1, t2, false));
    ADJ_OK(rhot_t(k, ztb, false));
  }
  // guess: dt z_t^0 = co . (z, h1, h2, h3)
  if (!zero_guess) {
    axpy(a, ztb, zb, co[0] / dt);
    for (int h = 0; h < 3; ++h)
      if (g->z_hist[h]) {
        axpy(a, ztb, static_cast<double2*>(g->z_hist[h]), co[h + 1] / dt, AM_ONE, false);
        herm(static_cast<double2*>(g->z_hist[h]), false, false);
      }
  } else {
    for (int h = 0; h < 3; ++h)
      if (g->z_hist[h]) clear(a, static_cast<double2*>(g->z_hist[h]));
  }
  // R_z = P_N^{-1} Fwd(R): R_bar on the grid, then the pointwise transpose
  proj_t(a, 2, rzb, t1);
  ADJ_OK(fwd_t(a, t1, pt[0]));
  {
    AdjPointArgs A{};
    A.zp = zp;
    for (int i = 0; i < 3; ++i) A.g[i] = gz[i], A.m[i] = mdp[i], A.out[i] = pt[1 + i], A.gb[i] = gb[i];
    A.lap = lap;
    A.in[0] = pt[0];
    A.zpb = zpb;
    A.lapb = lapb;
    pointwise(AP_RZ_T, A);
  }
  ADJ_OK(phys_to_coef_t(a, pt[1], EV_E0, mdb1, t1, t2, true));
  ADJ_OK(phys_to_coef_t(a, pt[2], EV_F0, mdb2, t1, t2, true));
  ADJ_OK(phys_to_coef_t(a, pt[3], EV_E0, mdb3, t1, t2, true));
  // z on the grid: zp = Inv E0 z, g = Inv(i k1 E0 z), Inv E1 z, Inv(i k3 E0 z), lap = Inv(E2 z - k^2 E0 z)
  ADJ_OK(phys_to_coef_t(a, zpb, EV_E0, zb, t1, t2, true));
  ADJ_OK(phys_to_coef_t(a, gb[0], EV_E0, zb, t1, t2, true, AM_NIK1));
  ADJ_OK(phys_to_coef_t(a, gb[1], EV_E1, zb, t1, t2, true));
  ADJ_OK(phys_to_coef_t(a, gb[2], EV_E0, zb, t1, t2, true, AM_NIK3));
  ADJ_OK(inv_t(a, lapb, t3));
  eval_t(a, EV_E2, t3, t2);
  axpy(a, t2, zb);
  axpy(a, t3, t3, -1.0, AM_KSQ, false);
  eval_t(a, EV_E0, t3, t2);
  axpy(a, t2, zb);
  // m^d^T: (phi2, Omega2, <m>1, <m>3) gradients, plus the direct paths X -> X_out
  double* m1bar_t = tmpv;
  double* m3bar_t = tmpv + n2;
  {
    double2* scr = a.c.at<double2>(p->ws.off_yt);
    hipLaunchKernelGGL(k_md_t, a.gC, dim3(kThreads), 0, s, p->D, mdb1, mdb2, mdb3, static_cast<double2*>(g->phi2),
                       static_cast<double2*>(g->omega2), m1bar_t, m3bar_t, scr);
  }
  axpy(a, cS(g->phi2_out), static_cast<double2*>(g->phi2));
  axpy(a, cS(g->omega2_out), static_cast<double2*>(g->omega2));
  herm(static_cast<double2*>(g->phi2), false, true);
  herm(static_cast<double2*>(g->omega2), false, true);
  vaxpy(1.0, m1bar_t, 1.0, g->m1bar_out, g->m1bar, false);
  vaxpy(1.0, m3bar_t, 1.0, g->m3bar_out, g->m3bar, false);
  herm(zb, false, false);
  axpy(a, zb, static_cast<double2*>(g->z), 1.0, AM_ONE, false);
  if (fa->stage == 1) {
    for (void* q : {g->rhs_phi2_prev, g->rhs_omega2_prev}) if (q) herm(static_cast<double2*>(q), false, true);
    if (g->zt_prev) herm(static_cast<double2*>(g->zt_prev), false, false);
  }
#undef ADJ_OK
  return hipGetLastError() == hipSuccess ? LMVD_OK : LMVD_EHIP;
}

}  // namespace lmvd

extern "C" {

lmvd_status lmvd_adjoint_sizes(lmvd_plan plan, int32_t kf, size_t* workspace_bytes) {
  if (!plan || !workspace_bytes) return LMVD_EINVAL;
  const int k = kf < 0 ? plan->H.cfg.kf : kf;
  if (k < 0 || k > 64) return LMVD_EINVAL;
  *workspace_bytes = lmvd::adjoint_layout(plan, k).bytes;
  return LMVD_OK;
}

lmvd_status lmvd_substep_adjoint(lmvd_plan plan, const lmvd_substep_args* a, const lmvd_substep_grads* g,
                                 void* workspace, void* stream) {
  if (!plan || !a || !g || !workspace) return LMVD_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return LMVD_EINVAL;
  if (a->stage != 0 && a->stage != 1) return LMVD_EINVAL;
  if (a->guess_mode != 0 && a->guess_mode != 1) return LMVD_EINVAL;
  const lmvd_config& cfg = plan->H.cfg;
  for (int k = 0; k < 3; ++k)
    if (cfg.mu_z[k] != 0.0 || cfg.rhoD_z[k] != 0.0) return LMVD_EUNSUPPORTED;
  if (cfg.rhoD_form != 0) return LMVD_EUNSUPPORTED;
  const int kf = a->kf < 0 ? cfg.kf : a->kf;
  if (kf < 0 || kf > 64) return LMVD_EINVAL;
  const void* need[] = {a->phi2, a->omega2, a->z, a->m1bar, a->m3bar, g->phi2_out, g->omega2_out, g->z_out,
                        g->m1bar_out, g->m3bar_out, g->rhs_phi2, g->rhs_omega2, g->zt, g->rhs_m1, g->rhs_m3,
                        g->phi2, g->omega2, g->z, g->m1bar, g->m3bar};
  for (const void* q : need)
    if (!q || !lmvd::aligned(q)) return LMVD_EINVAL;
  if (a->guess_mode == 0)
    for (int h = 0; h < 3; ++h)
      if (!a->z_hist[h]) return LMVD_EINVAL;
  if (hipSetDevice(plan->device) != hipSuccess) return LMVD_EHIP;
  return lmvd::run_substep_adjoint(plan, a, g, static_cast<char*>(workspace), static_cast<hipStream_t>(stream), kf);
}

}  // extern "C"
