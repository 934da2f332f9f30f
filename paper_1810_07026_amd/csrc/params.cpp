// Host-side reader of the AIREBO parameter file and builder of the spline
// coefficient tables uploaded to the GPU.
//
// The file holds knot data (values and first derivatives at integer knots for
// the bicubic P and tricubic pi^rc / T tables, with zero cross derivatives;
// value, first and second derivative at each knot of the angular functions g).
// Each spline is the Hermite interpolant of that data; here it is expanded
// into monomial coefficients per cell so that a kernel evaluates it with
// Horner's rule.  Functional form: Sec. 2.1.3 (b_ij, p_ij, pi^rc, pi^dh) and
// Sec. 2.1.2 (LJ switches) of "Optimizing AIREBO".
#include "params.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

namespace airebo {
namespace {

struct Rec { std::string key; std::vector<double> v; };

// Cubic Hermite basis on [0,1] in monomial form: [end][kind][power],
// kind 0 = value at that end, 1 = derivative at that end.
const double kCub[2][2][4] = {
    {{1, 0, -3, 2}, {0, 1, -2, 1}},
    {{0, 0, 3, -2}, {0, 0, -1, 1}},
};
// Quintic Hermite basis on [0,1]: value/derivative/second derivative at each end.
const double kQuin[2][3][6] = {
    {{1, 0, 0, -10, 15, -6}, {0, 1, 0, -6, 8, -3}, {0, 0, 0.5, -1.5, 1.5, -0.5}},
    {{0, 0, 0, 10, -15, 6}, {0, 0, 0, -4, 7, -3}, {0, 0, 0, 0.5, -1, 0.5}},
};

struct K3 { double f = 0, d[3] = {0, 0, 0}; bool set = false; };

bool make_gspline(const std::vector<std::vector<double>>& knots, GSpline& g, std::string& err) {
  if (knots.size() < 2 || knots.size() > (size_t)kMaxKnots) { err = "angular spline needs 2..8 knots"; return false; }
  std::memset(&g, 0, sizeof g);
  g.n = (int)knots.size();
  for (int m = 0; m < g.n; ++m) {
    g.x[m] = knots[m][0];
    if (m && !(g.x[m] > g.x[m - 1])) { err = "angular knots not increasing"; return false; }
  }
  for (int m = 0; m + 1 < g.n; ++m) {
    double h = g.x[m + 1] - g.x[m];
    g.inv_h[m] = 1.0 / h;
    const std::vector<double>* e[2] = {&knots[m], &knots[m + 1]};
    for (int p = 0; p < 6; ++p) {
      double c = 0;
      for (int end = 0; end < 2; ++end)
        c += (*e[end])[1] * kQuin[end][0][p] + h * (*e[end])[2] * kQuin[end][1][p] + h * h * (*e[end])[3] * kQuin[end][2][p];
      g.c[m][p] = c;
    }
  }
  return true;
}

}  // namespace

bool build_params(const char* path, DevParams& P, double* tri, std::string& err) {
  FILE* f = std::fopen(path, "rb");
  if (!f) { err = std::string("cannot open parameter file ") + path; return false; }
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  return build_params_text(text.data(), text.size(), P, tri, err);
}

bool build_params_text(const char* text, size_t len, DevParams& P, double* tri, std::string& err) {
  std::vector<Rec> recs;
  size_t pos = 0;
  while (pos < len) {
    size_t eol = pos;
    while (eol < len && text[eol] != '\n') ++eol;
    std::string line(text + pos, eol - pos);
    pos = eol + 1;
    size_t h = line.find('#');
    if (h != std::string::npos) line.resize(h);
    char* save = nullptr;
    char* tok = strtok_r(&line[0], " \t\r\n", &save);
    if (!tok) continue;
    Rec r;
    r.key = tok;
    while ((tok = strtok_r(nullptr, " \t\r\n", &save))) {
      char* end = nullptr;
      double v = std::strtod(tok, &end);
      if (end == tok || *end) { err = "non-numeric field in record " + r.key; return false; }
      r.v.push_back(v);
    }
    recs.push_back(r);
  }

  std::memset(&P, 0, sizeof P);
  std::map<std::string, double> sc;
  std::vector<std::vector<double>> gC, gam, gH;
  static K3 Pk[2][5][5];
  static K3 Tk[TRI_N][5][5][9];
  std::memset(Pk, 0, sizeof Pk);
  for (int t = 0; t < TRI_N; ++t)
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b)
        for (int c = 0; c < 9; ++c) Tk[t][a][b][c] = K3();
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < 5; ++a)
      for (int b = 0; b < 5; ++b) Pk[s][a][b] = K3();

  auto set3 = [&](K3& k, double fv, double d0, double d1, double d2) -> bool {
    if (k.set) return false;
    k.set = true; k.f = fv; k.d[0] = d0; k.d[1] = d1; k.d[2] = d2;
    return true;
  };
  for (const Rec& r : recs) {
    const std::string& k = r.key;
    const std::vector<double>& v = r.v;
    if (k == "gC" || k == "gammaC" || k == "gH") {
      if (v.size() != 4) { err = "knot record " + k + " needs 4 numbers"; return false; }
      (k == "gC" ? gC : k == "gammaC" ? gam : gH).push_back(v);
    } else if (k == "P_CC" || k == "P_CH") {
      if (v.size() != 5) { err = k + " record needs 5 numbers"; return false; }
      int a = (int)v[0], b = (int)v[1];
      if (a != v[0] || b != v[1] || a < 0 || a > 4 || b < 0 || b > 4) { err = k + " knot index out of range"; return false; }
      if (!set3(Pk[k == "P_CH"][a][b], v[2], v[3], v[4], 0)) { err = "duplicate knot in " + k; return false; }
    } else if (k == "F_CC" || k == "F_CH" || k == "F_HH" || k == "T_CC") {
      if (v.size() != 7) { err = k + " record needs 7 numbers"; return false; }
      int a = (int)v[0], b = (int)v[1], c = (int)v[2];
      if (a != v[0] || b != v[1] || c != v[2] || a < 0 || a > 4 || b < 0 || b > 4 || c < 1 || c > 9) {
        err = k + " knot index out of range"; return false;
      }
      int t = k == "F_CC" ? TRI_FCC : k == "F_CH" ? TRI_FCH : k == "F_HH" ? TRI_FHH : TRI_TCC;
      if (!set3(Tk[t][a][b][c - 1], v[3], v[4], v[5], v[6])) { err = "duplicate knot in " + k; return false; }
      if (t != TRI_FCH) {          // symmetric in (N_ij, N_ji): mirror
        if (a > b) { err = k + " records must have i <= j"; return false; }
        if (a != b) {
          if (!set3(Tk[t][b][a][c - 1], v[3], v[5], v[4], v[6])) { err = "duplicate mirrored knot in " + k; return false; }
        } else if (v[4] != v[5]) {
          err = k + " diagonal knot needs equal derivatives in i and j"; return false;
        }
      }
    } else {
      if (v.size() != 1) { err = "scalar record " + k + " needs 1 number"; return false; }
      sc[k] = v[0];
    }
  }
  auto need = [&](const std::string& name, double& out) -> bool {
    auto it = sc.find(name);
    if (it == sc.end()) { err = "missing parameter " + name; return false; }
    out = it->second;
    return true;
  };
  const char* pn[3] = {"CC", "CH", "HH"};
  for (int p = 0; p < 3; ++p) {
    std::string s = pn[p];
    if (!need("R1_" + s, P.R1[p]) || !need("R2_" + s, P.R2[p]) || !need("Q_" + s, P.Q[p]) || !need("A_" + s, P.A[p]) ||
        !need("alpha_" + s, P.alpha[p]) || !need("bmin_" + s, P.bmin[p]) || !need("bmax_" + s, P.bmax[p]))
      return false;
    for (int m = 0; m < 3; ++m)
      if (!need("B" + std::to_string(m + 1) + "_" + s, P.B[p][m]) || !need("beta" + std::to_string(m + 1) + "_" + s, P.beta[p][m]))
        return false;
    if (!(P.R1[p] > 0 && P.R2[p] > P.R1[p])) { err = "REBO cutoffs must satisfy 0 < R1 < R2"; return false; }
    if (!(P.bmax[p] > P.bmin[p])) { err = "bmax must exceed bmin"; return false; }
    P.inv_db[p] = 1.0 / (P.bmax[p] - P.bmin[p]);
    P.inv_dR[p] = 1.0 / (P.R2[p] - P.R1[p]);
  }
  double sCC, sHH, eCC, eHH, cut, bs;
  if (!need("rho_CH", P.rho[0]) || !need("rho_HH", P.rho[1]) || !need("lambda_pref", P.lambda_pref) ||
      !need("gC_blend_lo", P.gC_lo) || !need("gC_blend_hi", P.gC_hi) || !need("conj_lo", P.conj_lo) ||
      !need("conj_hi", P.conj_hi) || !need("dihedral_guard_on", P.guard_on) || !need("dihedral_guard_off", P.guard_off) ||
      !need("tors_eps_CCCC", P.tors_eps[0]) || !need("tors_eps_HCCC", P.tors_eps[1]) ||
      !need("tors_eps_HCCH", P.tors_eps[2]) || !need("sigma_CC", sCC) || !need("sigma_HH", sHH) ||
      !need("epsilon_CC", eCC) || !need("epsilon_HH", eHH) || !need("LJ_cut_sigma", cut) ||
      !need("LJ_switch_width", P.lj_sw) || !need("bstar_use_R1", bs))
    return false;
  if (!(P.gC_hi > P.gC_lo && P.conj_hi > P.conj_lo && P.guard_off > P.guard_on && P.lj_sw > 0)) {
    err = "switch ranges must be increasing"; return false;
  }
  P.bstar_use_R1 = bs != 0;
  P.inv_guard = 1.0 / (P.guard_off - P.guard_on);
  P.inv_lj_sw = 1.0 / P.lj_sw;
  // Morse pair term of AIREBO-M: all nine records or none
  P.morse_ok = 0;
  if (sc.count("morse_eps_CC")) {
    for (int p = 0; p < 3; ++p) {
      std::string t = pn[p];
      if (!need("morse_eps_" + t, P.m_eps[p]) || !need("morse_re_" + t, P.m_re[p]) ||
          !need("morse_alpha_" + t, P.m_alpha[p]))
        return false;
      if (!(P.m_eps[p] > 0 && P.m_re[p] > 0 && P.m_alpha[p] > 0)) { err = "Morse parameters must be positive"; return false; }
    }
    P.morse_ok = 1;
  }
  P.sigma[0] = sCC; P.sigma[2] = sHH; P.sigma[1] = 0.5 * (sCC + sHH);   // Lorentz-Berthelot
  P.eps[0] = eCC; P.eps[2] = eHH; P.eps[1] = std::sqrt(eCC * eHH);
  P.rc_max = 0; P.R2max = 0;
  for (int p = 0; p < 3; ++p) {
    P.rc[p] = cut * P.sigma[p];
    P.rc2[p] = P.rc[p] * P.rc[p];
    P.rljmax[p] = std::pow(2.0, 1.0 / 6.0) * P.sigma[p];
    P.inv_rlj[p] = 1.0 / (P.rljmax[p] - P.sigma[p]);
    P.rc_max = std::fmax(P.rc_max, P.rc[p]);
    P.R2max = std::fmax(P.R2max, P.R2[p]);
    if (P.rc[p] - P.lj_sw < P.rljmax[p]) { err = "LJ switch region overlaps the bond-order switch"; return false; }
  }
  P.r_conn = 3.0 * P.R2max;
  P.knot_delta = 1e-3;
  for (int p = 0; p < 3; ++p)
    if (P.rljmax[p] >= P.r_conn) { err = "LJ bond-order switch must lie inside three REBO bond lengths"; return false; }

  if (!make_gspline(gC, P.gC, err) || !make_gspline(gH, P.gH, err) || !make_gspline(gam, P.gammaC, err)) return false;
  if (std::fabs(P.gammaC.x[P.gammaC.n - 1] - P.gC.x[P.gC.n - 1]) > 1e-12) { err = "gammaC must end where gC ends"; return false; }

  // bicubic P: [s_j][cell NC][cell NH]
  for (int s = 0; s < 2; ++s)
    for (int cx = 0; cx < 4; ++cx)
      for (int cy = 0; cy < 4; ++cy)
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            double c = 0;
            for (int ex = 0; ex < 2; ++ex)
              for (int ey = 0; ey < 2; ++ey) {
                const K3& q = Pk[s][cx + ex][cy + ey];
                c += q.f * kCub[ex][0][a] * kCub[ey][0][b] + q.d[0] * kCub[ex][1][a] * kCub[ey][0][b] +
                     q.d[1] * kCub[ex][0][a] * kCub[ey][1][b];
              }
            P.Pc[s][cx][cy][a * 4 + b] = c;
          }
  // tricubic tables
  for (int t = 0; t < TRI_N; ++t)
    for (int cx = 0; cx < 4; ++cx)
      for (int cy = 0; cy < 4; ++cy)
        for (int cz = 0; cz < 8; ++cz) {
          int cell = (cx * 4 + cy) * 8 + cz;
          double* out = tri + ((size_t)t * kTriCells + cell) * kTriCoef;
          bool nz = false;
          for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
              for (int c = 0; c < 4; ++c) {
                double v = 0;
                for (int ex = 0; ex < 2; ++ex)
                  for (int ey = 0; ey < 2; ++ey)
                    for (int ez = 0; ez < 2; ++ez) {
                      const K3& q = Tk[t][cx + ex][cy + ey][cz + ez];
                      v += q.f * kCub[ex][0][a] * kCub[ey][0][b] * kCub[ez][0][c] +
                           q.d[0] * kCub[ex][1][a] * kCub[ey][0][b] * kCub[ez][0][c] +
                           q.d[1] * kCub[ex][0][a] * kCub[ey][1][b] * kCub[ez][0][c] +
                           q.d[2] * kCub[ex][0][a] * kCub[ey][0][b] * kCub[ez][1][c];
                    }
                out[(a * 4 + b) * 4 + c] = v;
                nz = nz || v != 0.0;
              }
          P.tri_nz[t][cell] = nz;
        }
  return true;
}

}  // namespace airebo
