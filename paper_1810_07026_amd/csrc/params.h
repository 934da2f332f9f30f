// Device-side parameter block of the AIREBO library and its host builder.
//
// Scalars and the small spline coefficient tables live in one POD struct that
// kernels read through a pointer (uniform loads).  The tricubic tables
// (pi^rc F_CC, F_CH, F_HH and the dihedral prefactor T_CC) are large and live
// in a separate device array referenced by `tri`.
//
// All splines are stored as monomial coefficients in the local coordinate of
// their cell: quintic pieces for the angular functions g (6 per interval),
// bicubic for P (16 per unit cell), tricubic for F and T (64 per unit cell).
#pragma once
#include <string>

namespace airebo {

constexpr int kMaxKnots = 8;

struct GSpline {
  int n;                        // number of knots
  double x[kMaxKnots];          // knot positions (cos theta)
  double c[kMaxKnots - 1][6];   // per interval: value = sum_m c[m] t^m, t = (x - x0)/h
  double inv_h[kMaxKnots - 1];
};

// Tricubic table index
enum { TRI_FCC = 0, TRI_FCH = 1, TRI_FHH = 2, TRI_TCC = 3, TRI_N = 4 };
// Tricubic grid: N_ij, N_ji in [0,4] (4 cells each), Nconj in [1,9] (8 cells)
constexpr int kTriCells = 4 * 4 * 8;
constexpr int kTriCoef = 64;

struct DevParams {
  // species-pair index p = s_i + s_j: CC = 0, CH = 1, HH = 2
  double R1[3], R2[3], inv_dR[3];
  double Q[3], A[3], alpha[3], B[3][3], beta[3][3];
  double rho[2];                // rho_{sH}, s = C, H
  double lambda_pref;
  double gC_lo, gC_hi, conj_lo, conj_hi;
  GSpline gC, gammaC, gH;
  double Pc[2][4][4][16];       // [s_j][cNC][cNH][a*4+b]: sum c_ab tC^a tH^b
  double guard_on, guard_off, inv_guard;   // inv_guard = 1 / (guard_off - guard_on)
  double tors_eps[3];           // by number of H among the two end atoms
  double sigma[3], eps[3], rc[3], rc2[3], rljmax[3], inv_rlj[3];
  double lj_sw, inv_lj_sw;
  double bmin[3], bmax[3], inv_db[3];   // inv_db = 1 / (bmax - bmin)
  int bstar_use_R1;
  double rc_max;                // largest LJ cutoff
  double r_conn;                // no path of three bonds reaches beyond this (3 max R2)
  double R2max;
  int morse_ok;                 // Morse records present (AIREBO-M)
  double m_eps[3], m_re[3], m_alpha[3];
  double knot_delta;            // FP32 spline arguments this close to a knot are evaluated in FP64
                                // (set per context: 1e-3 for mixed precision, negative for single)
  unsigned char tri_nz[TRI_N][kTriCells];   // cell has a non-zero coefficient
  const double* tri;            // device: [TRI_N][kTriCells][kTriCoef]
};

// Parse the parameter file and fill `P` (tri left null) and the host copy of
// the tricubic coefficients (TRI_N * kTriCells * kTriCoef doubles).
bool build_params(const char* path, DevParams& P, double* tri_host, std::string& err);
// The same from the file's text in memory (len bytes).
bool build_params_text(const char* text, size_t len, DevParams& P, double* tri_host, std::string& err);

}  // namespace airebo
