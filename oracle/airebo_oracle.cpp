// AIREBO reference evaluation on the CPU, in FP64 -- TEST INFRASTRUCTURE ONLY.
//
// This file is the oracle against which the GPU library is checked.  It is
// meant to be slow and obviously correct: every energy term is written out as
// its plain definition and forces are obtained by forward-mode automatic
// differentiation (dual numbers) of each term's energy with respect to the
// coordinates of the atoms that term reads.  No derivative is derived by hand
// here, so nothing about the gradient is shared with the GPU kernels.
//
// Only the tests, the smoke check and the CPU-baseline leg of the benchmark
// may load this library.  It shares no source with the GPU path; the two read
// the same parameter file, each with its own parser.
//
// Functional form (Hoehnerbach & Bientinesi, "Optimizing AIREBO", Sec. 2.1 and
// its subsections; detail from the AIREBO and second-generation REBO papers
// that it names as the authority):
//   E = sum_{i<j bonded} w_ij [V^R(r_ij) - b_ij V^A(r_ij)]           (Sec. 2.1.1, Alg. 1)
//     + sum_{i<j, k, l} w_ki w_ij w_jl V^tors(omega_kijl)            (Sec. 2.1.1, Alg. 2)
//     + sum_{i<j} [S(t_r) S(t_b(b*_ij)) + 1 - S(t_r)] C_ij V^LJ(r)  (Sec. 2.1.2, Alg. 3)
//   b_ij = (p_ij + p_ji)/2 + pi^rc_ij + pi^dh_ij                      (Sec. 2.1.3)
//   C_ij = 1 - max{w_ij, w_ik w_kj, w_ik w_kl w_lj}                    (Sec. 2.1.2)
//   F_a = -dE/dx_a                                                      (Sec. 2)
// Readings where the paper is silent or garbled (sum, not product, of p_ij and
// p_ji; the constant that replaces r_ij in b*; collinear guards; the LJ outer
// switch; path identity under periodic images) are listed with the parameter
// file and in the design notes of the repository.
//
// Parity status: every function here is pinned by the CPU tests (finite
// differences, invariances, closed-form special cases, knot reproduction,
// brute-force enumeration), except the numerical values of the parameter set
// itself, which cannot be checked against the primary publications here.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <type_traits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Dual numbers: value plus gradient over the ND active coordinates of the
// current term (3 per site).  ND is set per term.
// ---------------------------------------------------------------------------
constexpr int MAXD = 3 * 96;
thread_local int ND = 0;

struct D {
  double v;
  double g[MAXD];
  D() : v(0.0) { for (int i = 0; i < ND; ++i) g[i] = 0.0; }
  D(double c) : v(c) { for (int i = 0; i < ND; ++i) g[i] = 0.0; }
};
inline double val(double x) { return x; }
inline double val(const D& x) { return x.v; }

inline D operator+(const D& a, const D& b) { D r(a.v + b.v); for (int i = 0; i < ND; ++i) r.g[i] = a.g[i] + b.g[i]; return r; }
inline D operator-(const D& a, const D& b) { D r(a.v - b.v); for (int i = 0; i < ND; ++i) r.g[i] = a.g[i] - b.g[i]; return r; }
inline D operator-(const D& a) { D r(-a.v); for (int i = 0; i < ND; ++i) r.g[i] = -a.g[i]; return r; }
inline D operator*(const D& a, const D& b) { D r(a.v * b.v); for (int i = 0; i < ND; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i]; return r; }
inline D operator/(const D& a, const D& b) {
  D r(a.v / b.v);
  double ib = 1.0 / b.v;
  for (int i = 0; i < ND; ++i) r.g[i] = (a.g[i] - r.v * b.g[i]) * ib;
  return r;
}
inline D operator+(const D& a, double b) { D r = a; r.v += b; return r; }
inline D operator+(double a, const D& b) { return b + a; }
inline D operator-(const D& a, double b) { D r = a; r.v -= b; return r; }
inline D operator-(double a, const D& b) { D r = -b; r.v += a; return r; }
inline D operator*(const D& a, double b) { D r(a.v * b); for (int i = 0; i < ND; ++i) r.g[i] = a.g[i] * b; return r; }
inline D operator*(double a, const D& b) { return b * a; }
inline D operator/(const D& a, double b) { return a * (1.0 / b); }
inline D operator/(double a, const D& b) { return D(a) / b; }
// chain rule helper: f(a) with f'(a) = d
inline D apply(const D& a, double f, double d) { D r(f); for (int i = 0; i < ND; ++i) r.g[i] = d * a.g[i]; return r; }
inline D sqrt(const D& a) { double s = std::sqrt(a.v); return apply(a, s, 0.5 / s); }
inline D exp(const D& a) { double e = std::exp(a.v); return apply(a, e, e); }
inline D cos(const D& a) { return apply(a, std::cos(a.v), -std::sin(a.v)); }
inline D abs(const D& a) { return a.v >= 0.0 ? a : -a; }
using std::sqrt; using std::exp; using std::cos; using std::abs;

template <class T> struct V3 { T x, y, z; };
template <class T> V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> T norm(const V3<T>& a) { return sqrt(dot(a, a)); }

// ---------------------------------------------------------------------------
// Parameters (own parser of the shared text format).
// ---------------------------------------------------------------------------
struct Knot { double x, f, d1, d2; };
struct KnotData { double f = 0, dx = 0, dy = 0, dz = 0; bool set = false; };

struct Params {
  // species-pair index: CC = 0, CH = 1, HH = 2 (sum of species codes)
  double R1[3], R2[3], Q[3], A[3], alpha[3], B[3][3], beta[3][3];
  double rho[2];               // rho_{sH} for s = C, H (lambda term)
  double lambda_pref;
  double gC_lo, gC_hi, conj_lo, conj_hi;
  std::vector<Knot> gC, gammaC, gH;
  KnotData P[2][5][5];         // [s_j][nC][nH] for a carbon centre
  KnotData F[3][5][5][9];      // pi^rc [pair][Nij][Nji][Nconj-1]
  KnotData T[5][5][9];         // pi^dh prefactor, C-C only
  double guard_on, guard_off;
  double tors_eps[3];          // by number of H among the two end atoms
  double sigma[3], eps[3];
  double lj_cut_sigma, lj_sw;
  double bmin[3], bmax[3];
  int bstar_use_R1;
  double rc_max;               // max over pairs of lj_cut_sigma * sigma
  // AIREBO-M: Morse well depth, minimum and range per pair (optional records)
  bool morse_ok = false;
  double m_eps[3], m_re[3], m_alpha[3];
};

bool parse_params(const char* path, Params& P, std::string& err) {
  FILE* f = std::fopen(path, "r");
  if (!f) { err = std::string("cannot open ") + path; return false; }
  std::map<std::string, double> sc;
  char line[1024];
  std::vector<std::pair<std::string, std::vector<double>>> recs;
  while (std::fgets(line, sizeof line, f)) {
    char* h = std::strchr(line, '#');
    if (h) *h = 0;
    char* tok = std::strtok(line, " \t\r\n");
    if (!tok) continue;
    std::string key = tok;
    std::vector<double> v;
    while ((tok = std::strtok(nullptr, " \t\r\n"))) v.push_back(std::atof(tok));
    recs.push_back({key, v});
  }
  std::fclose(f);
  auto knot3 = [&](KnotData& kd, const std::vector<double>& v, size_t off, int nd) -> bool {
    if (kd.set) return false;
    kd.set = true;
    kd.f = v[off];
    kd.dx = v[off + 1];
    kd.dy = v[off + 2];
    kd.dz = nd == 3 ? v[off + 3] : 0.0;
    return true;
  };
  for (auto& r : recs) {
    const std::string& k = r.first;
    const std::vector<double>& v = r.second;
    if (k == "gC" || k == "gammaC" || k == "gH") {
      if (v.size() != 4) { err = "bad knot record " + k; return false; }
      Knot kn{v[0], v[1], v[2], v[3]};
      (k == "gC" ? P.gC : k == "gammaC" ? P.gammaC : P.gH).push_back(kn);
    } else if (k == "P_CC" || k == "P_CH") {
      if (v.size() != 5) { err = "bad record " + k; return false; }
      int a = (int)v[0], b = (int)v[1];
      if (a < 0 || a > 4 || b < 0 || b > 4) { err = "P index out of range"; return false; }
      if (!knot3(P.P[k == "P_CH"][a][b], v, 2, 2)) { err = "duplicate P knot"; return false; }
    } else if (k == "F_CC" || k == "F_CH" || k == "F_HH" || k == "T_CC") {
      if (v.size() != 7) { err = "bad record " + k; return false; }
      int a = (int)v[0], b = (int)v[1], c = (int)v[2];
      if (a < 0 || a > 4 || b < 0 || b > 4 || c < 1 || c > 9) { err = "tricubic index out of range"; return false; }
      KnotData (*tab)[5][9] = k == "T_CC" ? P.T : P.F[k == "F_CC" ? 0 : k == "F_CH" ? 1 : 2];
      if (!knot3(tab[a][b][c - 1], v, 3, 3)) { err = "duplicate tricubic knot " + k; return false; }
      bool mirror = (k != "F_CH") && a != b;
      if (mirror) {
        if (a > b) { err = "symmetric table records must have i <= j"; return false; }
        std::vector<double> m = {v[0], v[1], v[2], v[3], v[5], v[4], v[6]};
        if (!knot3(tab[b][a][c - 1], m, 3, 3)) { err = "duplicate mirrored knot"; return false; }
      } else if (k != "F_CH" && v[4] != v[5]) {
        err = "diagonal knot of a symmetric table needs dF/di == dF/dj"; return false;
      }
    } else {
      if (v.size() != 1) { err = "bad scalar record " + k; return false; }
      sc[k] = v[0];
    }
  }
  const char* pn[3] = {"CC", "CH", "HH"};
  auto get = [&](const std::string& name, double& out) -> bool {
    auto it = sc.find(name);
    if (it == sc.end()) { err = "missing scalar " + name; return false; }
    out = it->second;
    return true;
  };
  for (int p = 0; p < 3; ++p) {
    std::string s = pn[p];
    if (!get("R1_" + s, P.R1[p]) || !get("R2_" + s, P.R2[p]) || !get("Q_" + s, P.Q[p]) ||
        !get("A_" + s, P.A[p]) || !get("alpha_" + s, P.alpha[p]) || !get("bmin_" + s, P.bmin[p]) ||
        !get("bmax_" + s, P.bmax[p]))
      return false;
    for (int n = 0; n < 3; ++n) {
      if (!get("B" + std::to_string(n + 1) + "_" + s, P.B[p][n]) ||
          !get("beta" + std::to_string(n + 1) + "_" + s, P.beta[p][n]))
        return false;
    }
    if (!(P.R1[p] > 0 && P.R1[p] < P.R2[p])) { err = "cutoffs not ordered"; return false; }
  }
  double sCC, sHH, eCC, eHH;
  if (!get("rho_CH", P.rho[0]) || !get("rho_HH", P.rho[1]) || !get("lambda_pref", P.lambda_pref) ||
      !get("gC_blend_lo", P.gC_lo) || !get("gC_blend_hi", P.gC_hi) || !get("conj_lo", P.conj_lo) ||
      !get("conj_hi", P.conj_hi) || !get("dihedral_guard_on", P.guard_on) ||
      !get("dihedral_guard_off", P.guard_off) || !get("tors_eps_CCCC", P.tors_eps[0]) ||
      !get("tors_eps_HCCC", P.tors_eps[1]) || !get("tors_eps_HCCH", P.tors_eps[2]) ||
      !get("sigma_CC", sCC) || !get("sigma_HH", sHH) || !get("epsilon_CC", eCC) ||
      !get("epsilon_HH", eHH) || !get("LJ_cut_sigma", P.lj_cut_sigma) ||
      !get("LJ_switch_width", P.lj_sw))
    return false;
  double bs = 1;
  if (!get("bstar_use_R1", bs)) return false;
  P.bstar_use_R1 = (int)bs;
  // Morse records: all nine or none
  if (sc.count("morse_eps_CC")) {
    for (int p = 0; p < 3; ++p) {
      std::string t = pn[p];
      if (!get("morse_eps_" + t, P.m_eps[p]) || !get("morse_re_" + t, P.m_re[p]) ||
          !get("morse_alpha_" + t, P.m_alpha[p]))
        return false;
      if (!(P.m_eps[p] > 0 && P.m_re[p] > 0 && P.m_alpha[p] > 0)) { err = "Morse parameters must be positive"; return false; }
    }
    P.morse_ok = true;
  }
  // Lorentz-Berthelot mixing
  P.sigma[0] = sCC; P.sigma[2] = sHH; P.sigma[1] = 0.5 * (sCC + sHH);
  P.eps[0] = eCC; P.eps[2] = eHH; P.eps[1] = std::sqrt(eCC * eHH);
  P.rc_max = 0;
  for (int p = 0; p < 3; ++p) P.rc_max = std::max(P.rc_max, P.lj_cut_sigma * P.sigma[p]);
  auto sorted = [](const std::vector<Knot>& k) {
    for (size_t i = 1; i < k.size(); ++i) if (!(k[i].x > k[i - 1].x)) return false;
    return k.size() >= 2;
  };
  if (!sorted(P.gC) || !sorted(P.gammaC) || !sorted(P.gH)) { err = "angular knots not increasing"; return false; }
  if (P.guard_off <= P.guard_on || P.lj_sw <= 0) { err = "bad switch parameters"; return false; }
  return true;
}

// ---------------------------------------------------------------------------
// Switching functions.
// ---------------------------------------------------------------------------
// REBO bond weight: 1 below R1, 0 above R2, half-cosine between.
template <class T> T cutw(const T& r, double R1, double R2) {
  if (val(r) <= R1) return T(1.0);
  if (val(r) >= R2) return T(0.0);
  return 0.5 * (1.0 + cos(M_PI * (r - R1) / (R2 - R1)));
}
// The cubic switch S(t) of the LJ term: 1 for t <= 0, 0 for t >= 1.
template <class T> T Sw(const T& t) {
  if (val(t) <= 0.0) return T(1.0);
  if (val(t) >= 1.0) return T(0.0);
  return 1.0 - t * t * (3.0 - 2.0 * t);
}
// Half-cosine step from 1 (x <= lo) to 0 (x >= hi).
template <class T> T cosstep(const T& x, double lo, double hi) {
  if (val(x) <= lo) return T(1.0);
  if (val(x) >= hi) return T(0.0);
  return 0.5 * (1.0 + cos(M_PI * (x - lo) / (hi - lo)));
}
// Guard against (near-)collinear bond pairs in dihedral terms.
template <class T> T guard(const Params& P, const T& c) {
  T a = abs(c);
  return Sw((a - P.guard_on) / (P.guard_off - P.guard_on));
}

// ---------------------------------------------------------------------------
// Splines, evaluated from the knot data through the Hermite basis.
// ---------------------------------------------------------------------------
template <class T> T quintic(const std::vector<Knot>& k, T x) {
  if (val(x) <= k.front().x) x = T(k.front().x);
  if (val(x) >= k.back().x) x = T(k.back().x);
  size_t m = 0;
  while (m + 2 < k.size() && val(x) > k[m + 1].x) ++m;
  const Knot &a = k[m], &b = k[m + 1];
  double h = b.x - a.x;
  T t = (x - a.x) / h;
  T t2 = t * t, t3 = t2 * t, t4 = t3 * t, t5 = t4 * t;
  T H0 = 1.0 - 10.0 * t3 + 15.0 * t4 - 6.0 * t5;
  T H1 = t - 6.0 * t3 + 8.0 * t4 - 3.0 * t5;
  T H2 = 0.5 * t2 - 1.5 * t3 + 1.5 * t4 - 0.5 * t5;
  T H3 = 0.5 * t3 - t4 + 0.5 * t5;
  T H4 = -4.0 * t3 + 7.0 * t4 - 3.0 * t5;
  T H5 = 10.0 * t3 - 15.0 * t4 + 6.0 * t5;
  return a.f * H0 + (h * a.d1) * H1 + (h * h * a.d2) * H2 + (h * h * b.d2) * H3 + (h * b.d1) * H4 + b.f * H5;
}
// Cubic Hermite basis on the unit interval: value/derivative at end 0/1.
template <class T> T hv(int e, const T& t) { return e == 0 ? 1.0 - t * t * (3.0 - 2.0 * t) : t * t * (3.0 - 2.0 * t); }
template <class T> T hd(int e, const T& t) { return e == 0 ? t * (1.0 - t) * (1.0 - t) : t * t * (t - 1.0); }

template <class T> void cell_of(T& x, double lo, double hi, int& i0, T& t) {
  if (val(x) <= lo) x = T(lo);
  if (val(x) >= hi) x = T(hi);
  i0 = (int)std::floor(val(x) - lo);
  if (i0 > (int)(hi - lo) - 1) i0 = (int)(hi - lo) - 1;
  t = x - (lo + i0);
}
template <class T> T bicubic(const KnotData (&G)[5][5], T x, T y) {
  int ix, iy; T tx, ty;
  cell_of(x, 0.0, 4.0, ix, tx);
  cell_of(y, 0.0, 4.0, iy, ty);
  T s(0.0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const KnotData& q = G[ix + a][iy + b];
      s = s + q.f * hv(a, tx) * hv(b, ty) + q.dx * hd(a, tx) * hv(b, ty) + q.dy * hv(a, tx) * hd(b, ty);
    }
  return s;
}
template <class T> T tricubic(const KnotData (&G)[5][5][9], T x, T y, T z) {
  int ix, iy, iz; T tx, ty, tz;
  cell_of(x, 0.0, 4.0, ix, tx);
  cell_of(y, 0.0, 4.0, iy, ty);
  cell_of(z, 1.0, 9.0, iz, tz);
  T s(0.0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        const KnotData& q = G[ix + a][iy + b][iz + c];
        s = s + q.f * hv(a, tx) * hv(b, ty) * hv(c, tz) + q.dx * hd(a, tx) * hv(b, ty) * hv(c, tz) +
            q.dy * hv(a, tx) * hd(b, ty) * hv(c, tz) + q.dz * hv(a, tx) * hv(b, ty) * hd(c, tz);
      }
  return s;
}
// Angular function g of the centre species; for carbon blended over N_ij.
template <class T> T gfun(const Params& P, int si, const T& c, const T& Nij) {
  if (si == 1) return quintic(P.gH, c);
  T G = quintic(P.gC, c);
  if (val(c) <= P.gammaC.front().x) return G;
  T gam = quintic(P.gammaC, c);
  return G + cosstep(Nij, P.gC_lo, P.gC_hi) * (gam - G);
}

// ---------------------------------------------------------------------------
// System geometry and short (REBO) neighbour lists.
// ---------------------------------------------------------------------------
struct Sys {
  int n;
  std::vector<double> x;  // wrapped positions [n][3]
  const int* s;
  double L[3];
  int per[3];
};
struct Nb { int j; double d[3]; double r; };  // neighbour j at displacement d from i

inline void minimg(const Sys& S, double* d) {
  for (int c = 0; c < 3; ++c)
    if (S.per[c]) d[c] -= S.L[c] * std::nearbyint(d[c] / S.L[c]);
}

// Uniform cell grid over a periodic box (all dims periodic), cell side >= cut.
struct Grid {
  int nc[3];
  std::vector<std::vector<int>> cells;
  void build(const Sys& S, double cut) {
    for (int c = 0; c < 3; ++c) nc[c] = std::max(1, (int)std::floor(S.L[c] / cut));
    cells.assign((size_t)nc[0] * nc[1] * nc[2], {});
    for (int i = 0; i < S.n; ++i) cells[index(S, &S.x[3 * i])].push_back(i);
  }
  int coord(const Sys& S, double x, int c) const {
    int k = (int)std::floor(x / S.L[c] * nc[c]);
    return std::min(std::max(k, 0), nc[c] - 1);
  }
  size_t index(const Sys& S, const double* x) const {
    return ((size_t)coord(S, x[0], 0) * nc[1] + coord(S, x[1], 1)) * nc[2] + coord(S, x[2], 2);
  }
};

// Short neighbour lists N(i) = {k : r_ik < R2}, sorted by atom index.
void short_lists(const Params& P, const Sys& S, std::vector<std::vector<Nb>>& N) {
  N.assign(S.n, {});
  bool grid = S.per[0] && S.per[1] && S.per[2] && S.n > 2000;
  Grid G;
  if (grid) G.build(S, std::max(P.R2[0], std::max(P.R2[1], P.R2[2])) + 1e-9);
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < S.n; ++i) {
    auto consider = [&](int k) {
      if (k == i) return;
      double d[3] = {S.x[3 * k] - S.x[3 * i], S.x[3 * k + 1] - S.x[3 * i + 1], S.x[3 * k + 2] - S.x[3 * i + 2]};
      minimg(S, d);
      double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (r < P.R2[S.s[i] + S.s[k]]) N[i].push_back({k, {d[0], d[1], d[2]}, r});
    };
    if (!grid) {
      for (int k = 0; k < S.n; ++k) consider(k);
    } else {
      int ci[3];
      for (int c = 0; c < 3; ++c) ci[c] = G.coord(S, S.x[3 * i + c], c);
      std::vector<size_t> seen;
      for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
          for (int e = -1; e <= 1; ++e) {
            int q[3] = {ci[0] + a, ci[1] + b, ci[2] + e};
            for (int c = 0; c < 3; ++c) q[c] = ((q[c] % G.nc[c]) + G.nc[c]) % G.nc[c];
            size_t idx = ((size_t)q[0] * G.nc[1] + q[1]) * G.nc[2] + q[2];
            if (std::find(seen.begin(), seen.end(), idx) != seen.end()) continue;
            seen.push_back(idx);
            for (int k : G.cells[idx]) consider(k);
          }
    }
    std::sort(N[i].begin(), N[i].end(), [](const Nb& a, const Nb& b) { return a.j < b.j; });
  }
}

// ---------------------------------------------------------------------------
// Sites of one term: atoms with their positions relative to the term's
// first atom.  Each site contributes 3 dual coordinates.
// ---------------------------------------------------------------------------
struct Sites {
  std::vector<int> atom;
  std::vector<double> p;  // [nsite][3]
  int add(int a, const double* q) {
    for (size_t s = 0; s < atom.size(); ++s)
      if (atom[s] == a) return (int)s;  // unique image per atom within one term
    atom.push_back(a);
    p.insert(p.end(), q, q + 3);
    return (int)atom.size() - 1;
  }
  int n() const { return (int)atom.size(); }
};
inline void addv(const double* a, const double* b, double* o) { o[0] = a[0] + b[0]; o[1] = a[1] + b[1]; o[2] = a[2] + b[2]; }

// Topology of the bond-order of (i, j): neighbours of each end (excluding the
// other end) and, for each of those, its own neighbours (excluding the end).
struct Side {
  std::vector<int> k, ks;                 // site, species
  std::vector<std::vector<int>> m, ms;    // second shell per k: sites, species
};
struct BondTopo { int i = 0, j = 1; int si, sj; Side a, b; };

void side_topo(const std::vector<std::vector<Nb>>& N, const Sys& S, Sites& st, int ai, int aj,
               const double* pi, Side& sd) {
  for (const Nb& nk : N[ai]) {
    if (nk.j == aj) continue;
    double pk[3];
    addv(pi, nk.d, pk);
    sd.k.push_back(st.add(nk.j, pk));
    sd.ks.push_back(S.s[nk.j]);
    std::vector<int> ms, mss;
    for (const Nb& nm : N[nk.j]) {
      if (nm.j == ai) continue;
      double pm[3];
      addv(pk, nm.d, pm);
      ms.push_back(st.add(nm.j, pm));
      mss.push_back(S.s[nm.j]);
    }
    sd.m.push_back(ms);
    sd.ms.push_back(mss);
  }
}

template <class T> using Pos = std::vector<V3<T>>;

template <class T> Pos<T> seed(const Sites& st) {
  ND = 3 * st.n();
  Pos<T> X(st.n());
  for (int s = 0; s < st.n(); ++s) {
    T c[3];
    for (int d = 0; d < 3; ++d) {
      c[d] = T(st.p[3 * s + d]);
      if constexpr (std::is_same<T, D>::value) c[d].g[3 * s + d] = 1.0;
    }
    X[s] = {c[0], c[1], c[2]};
  }
  return X;
}

// Components of the bond order of (i, j), for inspection by tests.
template <class T> struct BO { T b, pij, pji, pirc, pidh, Nij, Nji, Nconj; };

// Bond order b_ij (Sec. 2.1.3).  With bstar, r_ij is replaced by R1_ij in the
// only place a bond length i-j enters (the lambda exponent); directions are kept.
template <class T>
BO<T> bond_order(const Params& P, const BondTopo& t, const Pos<T>& X, bool bstar) {
  const int pij = t.si + t.sj;
  V3<T> rij = sub(X[t.j], X[t.i]);
  T r = norm(rij);
  T r_lam = (bstar && P.bstar_use_R1) ? T(P.R1[pij]) : r;

  // One end (centre c, partner o): returns p, N^C, N^H, conj-sum.
  struct End { T p, N, conj; };
  auto end = [&](int c, int sc, int o, int so, const Side& sd, const V3<T>& rco, const T& rlam) -> End {
    T NC(0.0), NH(0.0);
    std::vector<T> w(sd.k.size());
    std::vector<V3<T>> rck(sd.k.size());
    std::vector<T> rk(sd.k.size());
    for (size_t q = 0; q < sd.k.size(); ++q) {
      rck[q] = sub(X[sd.k[q]], X[c]);
      rk[q] = norm(rck[q]);
      w[q] = cutw(rk[q], P.R1[sc + sd.ks[q]], P.R2[sc + sd.ks[q]]);
      if (sd.ks[q] == 0) NC = NC + w[q]; else NH = NH + w[q];
    }
    T N = NC + NH;
    T rco_n = norm(rco);
    T sum(0.0);
    for (size_t q = 0; q < sd.k.size(); ++q) {
      T cth = dot(rco, rck[q]) / (rco_n * rk[q]);
      T g = gfun(P, sc, cth, N);
      T lam(0.0);
      if (sc == 1) lam = P.lambda_pref * ((P.rho[sd.ks[q]] - rk[q]) - (P.rho[so] - rlam));
      sum = sum + w[q] * g * exp(lam);
    }
    T Pc(0.0);
    if (sc == 0) Pc = bicubic(P.P[so], NC, NH);
    T p = 1.0 / sqrt(1.0 + sum + Pc);
    T conj(0.0);
    for (size_t q = 0; q < sd.k.size(); ++q) {
      if (sd.ks[q] != 0) continue;
      T x(0.0);
      for (size_t u = 0; u < sd.m[q].size(); ++u) {
        T rkm = norm(sub(X[sd.m[q][u]], X[sd.k[q]]));
        x = x + cutw(rkm, P.R1[sd.ks[q] + sd.ms[q][u]], P.R2[sd.ks[q] + sd.ms[q][u]]);
      }
      conj = conj + w[q] * cosstep(x, P.conj_lo, P.conj_hi);
    }
    (void)o;
    return {p, N, conj};
  };
  V3<T> rji = sub(X[t.i], X[t.j]);
  End ei = end(t.i, t.si, t.j, t.sj, t.a, rij, r_lam);
  End ej = end(t.j, t.sj, t.i, t.si, t.b, rji, r_lam);
  T Nconj = 1.0 + ei.conj * ei.conj + ej.conj * ej.conj;
  T pirc;
  if (pij == 1) {  // C-H: arguments ordered carbon side first
    pirc = t.si == 0 ? tricubic(P.F[1], ei.N, ej.N, Nconj) : tricubic(P.F[1], ej.N, ei.N, Nconj);
  } else {
    pirc = tricubic(P.F[pij], ei.N, ej.N, Nconj);
  }
  T pidh(0.0);
  if (pij == 0) {
    T Tv = tricubic(P.T, ei.N, ej.N, Nconj);
    if (val(Tv) != 0.0) {
      T sum(0.0);
      for (size_t q = 0; q < t.a.k.size(); ++q) {
        V3<T> rik = sub(X[t.a.k[q]], X[t.i]);
        T wik = cutw(norm(rik), P.R1[t.si + t.a.ks[q]], P.R2[t.si + t.a.ks[q]]);
        T gi = guard(P, dot(rij, rik) / (r * norm(rik)));
        for (size_t u = 0; u < t.b.k.size(); ++u) {
          if (t.b.k[u] == t.a.k[q]) continue;  // l != k
          V3<T> rjl = sub(X[t.b.k[u]], X[t.j]);
          T wjl = cutw(norm(rjl), P.R1[t.sj + t.b.ks[u]], P.R2[t.sj + t.b.ks[u]]);
          T gj = guard(P, dot(rji, rjl) / (r * norm(rjl)));
          if (val(gi) == 0.0 || val(gj) == 0.0) continue;
          V3<T> e1 = cross(rji, rik), e2 = cross(rij, rjl);
          T cosT = dot(e1, e2) / (norm(e1) * norm(e2));
          sum = sum + (1.0 - cosT * cosT) * wik * wjl * gi * gj;
        }
      }
      pidh = Tv * sum;
    }
  }
  T b = 0.5 * (ei.p + ej.p) + pirc + pidh;
  return {b, ei.p, ej.p, pirc, pidh, ei.N, ej.N, Nconj};
}

// REBO pair energy of a bond (Alg. 1 with the cutoff and sign reading).
template <class T> T rebo_energy(const Params& P, const BondTopo& t, const Pos<T>& X) {
  const int p = t.si + t.sj;
  T r = norm(sub(X[t.j], X[t.i]));
  T w = cutw(r, P.R1[p], P.R2[p]);
  T VR = (1.0 + P.Q[p] / r) * P.A[p] * exp(-P.alpha[p] * r);
  T VA(0.0);
  for (int n = 0; n < 3; ++n)
    if (P.B[p][n] != 0.0) VA = VA + P.B[p][n] * exp(-P.beta[p][n] * r);
  BO<T> bo = bond_order(P, t, X, false);
  return w * (VR - bo.b * VA);
}

// Explicit torsion of one dihedral k-i-j-l (Alg. 2).  Sites 0..3 = k, i, j, l.
template <class T> T torsion_energy(const Params& P, const int sp[4], const Pos<T>& X) {
  V3<T> rik = sub(X[0], X[1]), rij = sub(X[2], X[1]), rjl = sub(X[3], X[2]), rji = sub(X[1], X[2]);
  T dik = norm(rik), dij = norm(rij), djl = norm(rjl);
  T w = cutw(dik, P.R1[sp[0] + sp[1]], P.R2[sp[0] + sp[1]]) * cutw(dij, P.R1[sp[1] + sp[2]], P.R2[sp[1] + sp[2]]) *
        cutw(djl, P.R1[sp[2] + sp[3]], P.R2[sp[2] + sp[3]]);
  T gi = guard(P, dot(rij, rik) / (dij * dik));
  T gj = guard(P, dot(rji, rjl) / (dij * djl));
  if (val(gi) == 0.0 || val(gj) == 0.0) return T(0.0);
  // normals of the planes (k,i,j) and (i,j,l): trans = 180 degrees
  V3<T> b1 = sub(X[1], X[0]), b2 = rij, b3 = rjl;
  V3<T> n1 = cross(b1, b2), n2 = cross(b2, b3);
  T cosw = dot(n1, n2) / (norm(n1) * norm(n2));
  T h = 0.5 * (1.0 + cosw);
  T h5 = h * h * h * h * h;
  double eps = P.tors_eps[sp[0] + sp[3]];
  return w * gi * gj * eps * ((256.0 / 405.0) * h5 - 0.1);
}

// ---------------------------------------------------------------------------
// LJ pair with C_ij and the bond-order switch (Alg. 3).
// ---------------------------------------------------------------------------
struct Path { int len; int a[4]; double p[4][3]; double prod; };  // sites along i .. j

// Best connection i -> j (the image of j at displacement dij), exhaustive over
// direct, one- and two-intermediate paths in a fixed order; the first maximum wins.
Path best_path(const Params& P, const Sys& S, const std::vector<std::vector<Nb>>& N, int i, int j,
               const double* dij, double rij) {
  Path best{0, {}, {}, 0.0};
  auto same_site = [&](const double* q) {
    return std::fabs(q[0] - dij[0]) + std::fabs(q[1] - dij[1]) + std::fabs(q[2] - dij[2]) < 1e-6;
  };
  const double o[3] = {0, 0, 0};
  // direct
  double w = cutw(rij, P.R1[S.s[i] + S.s[j]], P.R2[S.s[i] + S.s[j]]);
  if (w > best.prod) {
    best = {2, {i, j}, {}, w};
    std::memcpy(best.p[0], o, sizeof o); std::memcpy(best.p[1], dij, 3 * sizeof(double));
  }
  for (const Nb& k : N[i]) {
    if (k.j == j) continue;
    for (const Nb& kj : N[k.j]) {
      if (kj.j != j) continue;
      double q[3]; addv(k.d, kj.d, q);
      if (!same_site(q)) continue;
      double prod = cutw(k.r, P.R1[S.s[i] + S.s[k.j]], P.R2[S.s[i] + S.s[k.j]]) *
                    cutw(kj.r, P.R1[S.s[k.j] + S.s[j]], P.R2[S.s[k.j] + S.s[j]]);
      if (prod > best.prod) {
        best = {3, {i, k.j, j}, {}, prod};
        std::memcpy(best.p[0], o, sizeof o); std::memcpy(best.p[1], k.d, sizeof k.d); std::memcpy(best.p[2], q, sizeof q);
      }
    }
  }
  for (const Nb& k : N[i]) {
    if (k.j == j) continue;
    for (const Nb& l : N[k.j]) {
      if (l.j == i || l.j == j) continue;
      for (const Nb& lj : N[l.j]) {
        if (lj.j != j) continue;
        double pl[3], q[3]; addv(k.d, l.d, pl); addv(pl, lj.d, q);
        if (!same_site(q)) continue;
        double prod = cutw(k.r, P.R1[S.s[i] + S.s[k.j]], P.R2[S.s[i] + S.s[k.j]]) *
                      cutw(l.r, P.R1[S.s[k.j] + S.s[l.j]], P.R2[S.s[k.j] + S.s[l.j]]) *
                      cutw(lj.r, P.R1[S.s[l.j] + S.s[j]], P.R2[S.s[l.j] + S.s[j]]);
        if (prod > best.prod) {
          best = {4, {i, k.j, l.j, j}, {}, prod};
          std::memcpy(best.p[0], o, sizeof o); std::memcpy(best.p[1], k.d, sizeof k.d);
          std::memcpy(best.p[2], pl, sizeof pl); std::memcpy(best.p[3], q, sizeof q);
        }
      }
    }
  }
  return best;
}

struct LJStat { long long in_cut = 0, cij0 = 0, need_b = 0, dsb = 0; };

// ---------------------------------------------------------------------------
// Accumulators.
// ---------------------------------------------------------------------------
struct Acc {
  std::vector<double> F;
  double E[4] = {0, 0, 0, 0};  // total, REBO, LJ, torsion
  double W[6] = {0, 0, 0, 0, 0, 0};
  LJStat st;
  long long nbonds = 0, ndihed = 0;
};

// Scatter -dE/dp of a dual energy onto atoms; virial sum_s p_s (x) F_s.
void scatter(const Sites& st, const D& E, Acc& acc, int term) {
  acc.E[term] += E.v;
  for (int s = 0; s < st.n(); ++s) {
    double f[3] = {-E.g[3 * s], -E.g[3 * s + 1], -E.g[3 * s + 2]};
    int a = st.atom[s];
    for (int c = 0; c < 3; ++c) acc.F[3 * a + c] += f[c];
    const double* p = &st.p[3 * s];
    acc.W[0] += p[0] * f[0]; acc.W[1] += p[1] * f[1]; acc.W[2] += p[2] * f[2];
    acc.W[3] += p[0] * f[1]; acc.W[4] += p[0] * f[2]; acc.W[5] += p[1] * f[2];
  }
}

void bond_topo(const std::vector<std::vector<Nb>>& N, const Sys& S, int i, int j, const double* dij,
               Sites& st, BondTopo& t) {
  const double o[3] = {0, 0, 0};
  t.i = st.add(i, o);
  t.j = st.add(j, dij);
  t.si = S.s[i];
  t.sj = S.s[j];
  side_topo(N, S, st, i, j, o, t.a);
  side_topo(N, S, st, j, i, dij, t.b);
}

void do_bond(const Params& P, const Sys& S, const std::vector<std::vector<Nb>>& N, int i, const Nb& nj,
             int mask, Acc& acc) {
  int j = nj.j;
  acc.nbonds++;
  if (mask & 1) {
    Sites st;
    BondTopo t;
    bond_topo(N, S, i, j, nj.d, st, t);
    if (st.n() * 3 > MAXD) { std::fprintf(stderr, "oracle: bond term too large\n"); std::abort(); }
    Pos<D> X = seed<D>(st);
    scatter(st, rebo_energy(P, t, X), acc, 1);
  }
  if ((mask & 4) && S.s[i] == 0 && S.s[j] == 0) {
    for (const Nb& k : N[i]) {
      if (k.j == j) continue;
      for (const Nb& l : N[j]) {
        if (l.j == i || l.j == k.j) continue;
        acc.ndihed++;
        Sites st;
        const double o[3] = {0, 0, 0};
        double pl[3]; addv(nj.d, l.d, pl);
        st.atom = {k.j, i, j, l.j};
        st.p = {k.d[0], k.d[1], k.d[2], o[0], o[1], o[2], nj.d[0], nj.d[1], nj.d[2], pl[0], pl[1], pl[2]};
        int sp[4] = {S.s[k.j], S.s[i], S.s[j], S.s[l.j]};
        Pos<D> X = seed<D>(st);
        scatter(st, torsion_energy(P, sp, X), acc, 3);
      }
    }
  }
}

// The van der Waals pair term (Sec. 2.1.2): C_ij, the S_r / S_b blend and the
// outer cutoff switch multiply V(r), which is Lennard-Jones, or with `morse`
// the Morse form of the AIREBO-M variant (Sec. 2.1.2), eps [e^{-2a(r-re)} - 2 e^{-a(r-re)}].
void do_lj(const Params& P, const Sys& S, const std::vector<std::vector<Nb>>& N, int i, int j,
           const double* dij, double r, bool morse, Acc& acc) {
  const int p = S.s[i] + S.s[j];
  const double sig = P.sigma[p], eps = P.eps[p], rc = P.lj_cut_sigma * sig;
  if (r >= rc) return;
  acc.st.in_cut++;
  Path best = best_path(P, S, N, i, j, dij, r);
  if (best.prod >= 1.0) { acc.st.cij0++; return; }
  double tr = (r - sig) / (std::pow(2.0, 1.0 / 6.0) * sig - sig);
  bool need_b = tr < 1.0;
  Sites st;
  const double o[3] = {0, 0, 0};
  int si = st.add(i, o), sj = st.add(j, dij);
  std::vector<int> ps;
  for (int q = 0; q < best.len; ++q) ps.push_back(st.add(best.a[q], best.p[q]));
  BondTopo t;
  if (need_b) {
    acc.st.need_b++;
    t.i = si; t.j = sj; t.si = S.s[i]; t.sj = S.s[j];
    side_topo(N, S, st, i, j, o, t.a);
    side_topo(N, S, st, j, i, dij, t.b);
  }
  if (st.n() * 3 > MAXD) { std::fprintf(stderr, "oracle: LJ term too large\n"); std::abort(); }
  Pos<D> X = seed<D>(st);
  D rr = norm(sub(X[sj], X[si]));
  D prod(0.0);
  if (best.len > 0) {
    prod = D(1.0);
    for (int q = 0; q + 1 < best.len; ++q) {
      int a = ps[q], b = ps[q + 1];
      prod = prod * cutw(norm(sub(X[b], X[a])), P.R1[S.s[best.a[q]] + S.s[best.a[q + 1]]],
                         P.R2[S.s[best.a[q]] + S.s[best.a[q + 1]]]);
    }
  }
  D C = 1.0 - prod;
  D Sr = Sw((rr - sig) / (std::pow(2.0, 1.0 / 6.0) * sig - sig));
  D Qf(1.0);
  if (need_b) {
    BO<D> bo = bond_order(P, t, X, true);
    D tb = (bo.b - P.bmin[p]) / (P.bmax[p] - P.bmin[p]);
    if (tb.v > 0.0 && tb.v < 1.0) acc.st.dsb++;
    Qf = Sr * Sw(tb) + 1.0 - Sr;
  }
  D VLJ;
  if (morse) {
    D ex = exp(-P.m_alpha[p] * (rr - P.m_re[p]));
    VLJ = P.m_eps[p] * (ex * ex - 2.0 * ex);
  } else {
    D sr6 = D(sig) / rr;
    sr6 = sr6 * sr6 * sr6;
    sr6 = sr6 * sr6;
    VLJ = 4.0 * eps * (sr6 * sr6 - sr6);
  }
  D Scut = Sw((rr - (rc - P.lj_sw)) / P.lj_sw);
  scatter(st, Qf * C * VLJ * Scut, acc, 2);
}

// LJ pairs of atom i: j > i (all images), or, in selected mode, also j < i
// when j lies outside the near set.  Brute force with explicit image shifts.
template <class F> void lj_pairs_of(const Sys& S, double rc, int i, const Grid* G, F&& fn) {
  auto emit = [&](int j, double* d) {
    double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r < rc) fn(j, d, r);
  };
  if (!G) {
    int m[3];
    for (int c = 0; c < 3; ++c) m[c] = S.per[c] ? (int)std::ceil(rc / S.L[c]) : 0;
    for (int j = 0; j < S.n; ++j) {
      if (j == i) continue;
      for (int a = -m[0]; a <= m[0]; ++a)
        for (int b = -m[1]; b <= m[1]; ++b)
          for (int e = -m[2]; e <= m[2]; ++e) {
            double d[3] = {S.x[3 * j] - S.x[3 * i] + a * S.L[0], S.x[3 * j + 1] - S.x[3 * i + 1] + b * S.L[1],
                           S.x[3 * j + 2] - S.x[3 * i + 2] + e * S.L[2]};
            emit(j, d);
          }
    }
    return;
  }
  int ci[3];
  for (int c = 0; c < 3; ++c) ci[c] = G->coord(S, S.x[3 * i + c], c);
  size_t seen[27];
  int nseen = 0;
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b)
      for (int e = -1; e <= 1; ++e) {
        int q[3] = {ci[0] + a, ci[1] + b, ci[2] + e};
        for (int c = 0; c < 3; ++c) q[c] = ((q[c] % G->nc[c]) + G->nc[c]) % G->nc[c];
        size_t idx = ((size_t)q[0] * G->nc[1] + q[1]) * G->nc[2] + q[2];
        if (std::find(seen, seen + nseen, idx) != seen + nseen) continue;
        seen[nseen++] = idx;
        for (int j : G->cells[idx]) {
          if (j == i) continue;
          double d[3] = {S.x[3 * j] - S.x[3 * i], S.x[3 * j + 1] - S.x[3 * i + 1], S.x[3 * j + 2] - S.x[3 * i + 2]};
          minimg(S, d);
          emit(j, d);
        }
      }
}

struct Handle { Params P; };
thread_local std::string g_err;

int prepare(const Handle* H, int n, const double* x, const int* s, const double* box, const int* per, Sys& S) {
  const Params& P = H->P;
  if (n < 0 || !x || !s || !box || !per) { g_err = "bad argument"; return -1; }
  S.n = n; S.s = s;
  for (int c = 0; c < 3; ++c) {
    S.L[c] = box[c]; S.per[c] = per[c] ? 1 : 0;
    if (S.per[c] && !(box[c] >= std::max(12.0, P.rc_max))) { g_err = "periodic box side too small"; return -4; }
  }
  for (int i = 0; i < n; ++i) {
    if (s[i] != 0 && s[i] != 1) { g_err = "species must be 0 (C) or 1 (H)"; return -3; }
  }
  S.x.assign(x, x + 3 * (size_t)n);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      double& q = S.x[3 * i + c];
      if (!std::isfinite(q)) { g_err = "non-finite position"; return -5; }
      if (S.per[c]) { q -= S.L[c] * std::floor(q / S.L[c]); if (q >= S.L[c]) q -= S.L[c]; }
    }
  return 0;
}

}  // namespace

extern "C" {

const char* oracle_last_error() { return g_err.c_str(); }

void* oracle_params_new(const char* path) {
  Handle* h = new Handle();
  std::string err;
  if (!parse_params(path, h->P, err)) { g_err = err; delete h; return nullptr; }
  return h;
}
void oracle_params_free(void* h) { delete (Handle*)h; }
double oracle_rc_max(void* h) { return ((Handle*)h)->P.rc_max; }

// Energy, forces and virial.  sel == NULL: all terms, every output complete.
// sel != NULL: only terms whose support may contain a selected atom; forces
// are exact on the selected atoms only, energy and virial are partial.
// stats (may be NULL): [LJ pairs in cutoff, C_ij = 0, b* needed, dS_b != 0,
// bonds, dihedrals].
int oracle_compute(void* hp, int n, const double* x, const int* s, const double* box, const int* per,
                   int mask, const int* sel, int nsel, double* energy, double* forces, double* virial,
                   long long* stats, int nthreads) {
  const Handle* H = (const Handle*)hp;
  const Params& P = H->P;
  const bool morse = mask & 8;   // Morse in place of LJ (AIREBO-M)
  if (morse && !P.morse_ok) { g_err = "the parameter file has no Morse records"; return -2; }
  Sys S;
  int rc = prepare(H, n, x, s, box, per, S);
  if (rc) return rc;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  std::vector<std::vector<Nb>> N;
  short_lists(P, S, N);
  std::vector<char> nearm(n, sel ? 0 : 1);
  if (sel) {
    const double Dn = 6.5;  // covers every term support (<= 2 bonds from i or j)
#pragma omp parallel for schedule(static)
    for (int a = 0; a < n; ++a)
      for (int q = 0; q < nsel; ++q) {
        int b = sel[q];
        double d[3] = {S.x[3 * a] - S.x[3 * b], S.x[3 * a + 1] - S.x[3 * b + 1], S.x[3 * a + 2] - S.x[3 * b + 2]};
        minimg(S, d);
        if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < Dn * Dn) { nearm[a] = 1; break; }
      }
  }
  bool big = S.per[0] && S.per[1] && S.per[2] && S.L[0] >= 2 * P.rc_max + 1 && S.L[1] >= 2 * P.rc_max + 1 &&
             S.L[2] >= 2 * P.rc_max + 1 && n > 2000;
  Grid G;
  if (big) G.build(S, P.rc_max);
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  std::vector<Acc> accs(nt);
  for (auto& a : accs) a.F.assign(3 * (size_t)n, 0.0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < n; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    Acc& acc = accs[tid];
    if (mask & 5) {
      for (const Nb& nj : N[i]) {
        if (nj.j < i) continue;
        if (!nearm[i] && !nearm[nj.j]) continue;
        do_bond(P, S, N, i, nj, mask, acc);
      }
    }
    if ((mask & 2) && nearm[i]) {
      lj_pairs_of(S, P.rc_max, i, big ? &G : nullptr, [&](int j, double* d, double r) {
        if (j < i && nearm[j]) return;  // seen from j's side
        if (j < i) {  // canonical orientation i' < j'
          double dm[3] = {-d[0], -d[1], -d[2]};
          do_lj(P, S, N, j, i, dm, r, morse, acc);
        } else {
          do_lj(P, S, N, i, j, d, r, morse, acc);
        }
      });
    }
  }
  for (int c = 0; c < 4; ++c) energy[c] = 0;
  for (int c = 0; c < 6; ++c) virial[c] = 0;
  std::fill(forces, forces + 3 * (size_t)n, 0.0);
  long long st[6] = {0, 0, 0, 0, 0, 0};
  for (auto& a : accs) {
    for (size_t q = 0; q < a.F.size(); ++q) forces[q] += a.F[q];
    for (int c = 1; c < 4; ++c) energy[c] += a.E[c];
    for (int c = 0; c < 6; ++c) virial[c] += a.W[c];
    st[0] += a.st.in_cut; st[1] += a.st.cij0; st[2] += a.st.need_b; st[3] += a.st.dsb;
    st[4] += a.nbonds; st[5] += a.ndihed;
  }
  energy[0] = energy[1] + energy[2] + energy[3];
  if (stats) std::memcpy(stats, st, sizeof st);
  return 0;
}

// Spline evaluation for tests: which = 0 g_C(c, N), 1 g_H(c), 2 P_CC(nC, nH),
// 3 P_CH(nC, nH), 4 F_CC, 5 F_CH, 6 F_HH, 7 T_CC (3 arguments).  grad gets
// the partial derivatives with respect to each argument.
double oracle_spline(void* hp, int which, const double* args, double* grad) {
  const Params& P = ((Handle*)hp)->P;
  int na = which == 1 ? 1 : (which <= 3 ? 2 : 3);
  ND = na;
  D a[3];
  for (int q = 0; q < na; ++q) { a[q] = D(args[q]); a[q].g[q] = 1.0; }
  D r;
  switch (which) {
    case 0: r = gfun(P, 0, a[0], a[1]); break;
    case 1: r = gfun(P, 1, a[0], a[0]); break;
    case 2: r = bicubic(P.P[0], a[0], a[1]); break;
    case 3: r = bicubic(P.P[1], a[0], a[1]); break;
    case 4: r = tricubic(P.F[0], a[0], a[1], a[2]); break;
    case 5: r = tricubic(P.F[1], a[0], a[1], a[2]); break;
    case 6: r = tricubic(P.F[2], a[0], a[1], a[2]); break;
    default: r = tricubic(P.T, a[0], a[1], a[2]); break;
  }
  for (int q = 0; q < na; ++q) grad[q] = r.g[q];
  return r.v;
}

// Bond order of the pair (i, j) at displacement dij (the image of j), for
// tests.  out = [b, p_ij, p_ji, pi_rc, pi_dh, N_ij, N_ji, N_conj].
int oracle_bond_order(void* hp, int n, const double* x, const int* s, const double* box, const int* per,
                      int i, int j, const double* dij, int bstar, double* out) {
  const Handle* H = (const Handle*)hp;
  Sys S;
  int rc = prepare(H, n, x, s, box, per, S);
  if (rc) return rc;
  std::vector<std::vector<Nb>> N;
  short_lists(H->P, S, N);
  Sites st;
  BondTopo t;
  bond_topo(N, S, i, j, dij, st, t);
  ND = 0;
  Pos<double> X(st.n());
  for (int q = 0; q < st.n(); ++q) X[q] = {st.p[3 * q], st.p[3 * q + 1], st.p[3 * q + 2]};
  BO<double> b = bond_order(H->P, t, X, bstar != 0);
  double v[8] = {b.b, b.pij, b.pji, b.pirc, b.pidh, b.Nij, b.Nji, b.Nconj};
  std::memcpy(out, v, sizeof v);
  return 0;
}

// C_ij of the pair (i, j) at displacement dij, for tests.
double oracle_cij(void* hp, int n, const double* x, const int* s, const double* box, const int* per, int i,
                  int j, const double* dij) {
  const Handle* H = (const Handle*)hp;
  Sys S;
  if (prepare(H, n, x, s, box, per, S)) return std::nan("");
  std::vector<std::vector<Nb>> N;
  short_lists(H->P, S, N);
  double r = std::sqrt(dij[0] * dij[0] + dij[1] * dij[1] + dij[2] * dij[2]);
  return 1.0 - best_path(H->P, S, N, i, j, dij, r).prod;
}

// Velocity-Verlet NVE in metal units (A, fs, eV, amu).  thermo rows (every
// thermo_every steps and at the end): step, PE, KE, Etot, T, 0.
int oracle_nve(void* hp, int n, double* x, double* v, const int* s, const double* box, const int* per,
               const double* mass2, double dt, int nsteps, int thermo_every, double* thermo, int nthreads) {
  const double ftm = 1.0 / 103.642691;  // eV/(A amu) -> A/fs^2
  const double kB = 8.617333262e-5;
  std::vector<double> f(3 * (size_t)n);
  double e[4], w[6];
  int rc = oracle_compute(hp, n, x, s, box, per, 7, nullptr, 0, e, f.data(), w, nullptr, nthreads);
  if (rc) return rc;
  int row = 0;
  auto thermo_row = [&](int step) {
    double ke = 0;
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) ke += 0.5 * mass2[s[i]] * v[3 * i + c] * v[3 * i + c] / ftm;
    double T = n > 1 ? 2.0 * ke / ((3.0 * n - 3.0) * kB) : 0.0;
    double* r = thermo + 6 * row++;
    r[0] = step; r[1] = e[0]; r[2] = ke; r[3] = e[0] + ke; r[4] = T; r[5] = 0;
  };
  if (thermo && thermo_every > 0) thermo_row(0);
  for (int step = 1; step <= nsteps; ++step) {
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) {
        v[3 * i + c] += 0.5 * dt * f[3 * i + c] / mass2[s[i]] * ftm;
        x[3 * i + c] += dt * v[3 * i + c];
      }
    rc = oracle_compute(hp, n, x, s, box, per, 7, nullptr, 0, e, f.data(), w, nullptr, nthreads);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c) v[3 * i + c] += 0.5 * dt * f[3 * i + c] / mass2[s[i]] * ftm;
    if (thermo && thermo_every > 0 && (step % thermo_every == 0)) thermo_row(step);
  }
  return 0;
}

}  // extern "C"
