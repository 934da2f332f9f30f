// AIREBO energy / force / virial on MI355X (gfx950): kernels and the C ABI.
//
// Method: "Optimizing AIREBO" (Hoehnerbach & Bientinesi), Sec. 2.1:
//   REBO pair term with bond order b_ij (Alg. 1, Sec. 2.1.3), explicit torsion
//   (Alg. 2), Lennard-Jones with the C_ij connectivity switch and the modified
//   bond order b*_ij inside S_b (Alg. 3, Sec. 2.1.2); forces are the negative
//   gradient (Sec. 2), obtained here by a hand-written forward pass followed by
//   a reverse (chain-rule) pass per bond, the "AD without a tape" pattern the
//   paper describes for sums inside functions (Sec. 2).
//
// GPU design (one process, one device; everything stays in HBM):
//   rebuild (when any atom moved more than half the skin):
//     k_bin / k_fill             counting sort of atoms into cells >= half of LJ cutoff + skin
//     k_build                    one wavefront per atom: LJ list (with image shift
//                                codes) split into near pairs (within 3 max R2 +
//                                skin) and far pairs, and the intermediate REBO
//                                list (R2 + skin), filled by wave-ballot compaction
//                                (the vectorised list insertion of Sec. 4.1)
//   every step:
//     k_short                    exact short list from the intermediate list,
//                                w, dw/dr, coordination N^C, N^H; species-bucketed
//                                bond list (CC / CH / HH batches, Sec. 4.2)
//     k_lj                       one wavefront per atom: first the atom's path map
//                                in LDS (every atom reachable over <= 3 short bonds
//                                with its weight product and path: the reversed
//                                C_ij search of Sec. 4.3), then its near pairs:
//                                look up C_ij; pairs with 0 < C_ij < 1 or inside
//                                the S_r range are deferred to a queue (Sec. 4.3)
//     k_bstar                    one lane per queued pair: C_ij, b*, S_b, full
//                                gradient
//     k_ljf                      16 lanes per atom: the far pairs, plain LJ
//     k_bond                     one lane per bond: bond order, REBO pair term and
//                                torsion merged (Sec. 4.2), forward then reverse
//   The main stream runs k_short, k_lj, k_bstar; a second stream runs k_ljf
//   and k_bond beside them (launch_forces: the two schedules).
//   Forces are accumulated with hardware FP64 atomics (FP32 atomics into a
//   separate array in single precision, folded into the FP64 forces by
//   k_fold32); energies and the virial by block reduction followed by one
//   atomic per block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/airebo.h"
#include "params.h"

namespace airebo {

// Per-atom capacities.  The short and intermediate lists start at SCAP and
// ICAP entries per atom and grow (the evaluation or MD chunk is repeated)
// when an atom has more, up to SCAP_MAX and ICAP_MAX; their strides are
// Dev::scap and Dev::icap.
constexpr int SCAP = 8;          // short (REBO) neighbours per atom, initial
constexpr int SCAP_MAX = 32;     // path codes keep 5 bits per bond slot
constexpr int ICAP = 48;         // intermediate-list entries per atom, initial
constexpr int ICAP_MAX = 768;
constexpr int PCAP = 64;   // path-map candidates per atom (LDS, per wavefront); beyond: sequential C_ij search
constexpr int HCAP = 128;  // slots of the per-wavefront candidate lookup (2 x PCAP)
static_assert(PCAP == 64, "one path candidate per lane when the lookup is filled");
__device__ __forceinline__ int hslot(int a) { return (int)(((unsigned)a * 2654435761u) >> 25); }   // 7 bits
constexpr int LJ_BLOCK = 256;
constexpr int WAVE = 64;
// lanes per atom of the short-list kernel: an atom of a dense hydrocarbon has
// about a dozen intermediate entries, so each lane takes about two; with
// eight lanes the kernel's 110-register FP64 waves fit the device in one
// round (with sixteen they took two)
constexpr int SHORT_G = 8;

// flag bits
enum { F_REBUILD = 1, F_OV_SHORT = 2, F_OV_INT = 4, F_OV_LJ = 8, F_OV_PATH = 16, F_OV_BOND = 32, F_OV_QUEUE = 64,
       F_NONFINITE = 128, F_BADSPEC = 256, F_OV_NN = 512 };
// accumulator quantities; each lives in NSLOT copies (one per group of blocks,
// one cache line apart) that k_finish / k_thermo add up
enum { A_EREBO = 0, A_ETORS = 1, A_ELJ = 2, A_VIR = 3, A_NIN = 9, A_NC0 = 10, A_NDSB = 11, A_KE = 12, A_SPL = 13,
       A_SPL64 = 14, A_NSKIP = 15, A_NBSTAR = 16, A_NINF = 17, A_N = 24 };
// mixed precision: a spline argument within this distance of a knot is evaluated in FP64
// (single precision takes no such branch)
constexpr double KNOT_DELTA = 1e-3;
constexpr int NSLOT = 64;
// deferred-pair queue: NSEG segments with separate counters (QSTRIDE ints apart)
constexpr int NSEG = 64, QSTRIDE = 32;
// kernel ids for per-kernel timing
enum { K_LOAD, K_BIN, K_FILL, K_BUILD, K_ZERO, K_SHORT, K_BOND, K_LJ, K_BSTAR,
       K_FINISH, K_KICK_DRIFT, K_KICK, K_NN_ZERO, K_NN_ORDER, K_NN_DESC, K_NN_MLP, K_NN_FORCE, K_NN_PACK,
       K_NN_ENS, K_NN_DECIDE, K_FOLD32, K_LJF, K_COUNT };
const char* const kKernelNames[K_COUNT] = {
    "k_load", "k_bin", "k_fill", "k_build", "k_zero", "k_short", "k_bond",
    "k_lj", "k_bstar", "k_finish", "k_kick_drift", "k_kick", "nn_zero", "nn_order", "nn_desc",
    "nn_mlp", "nn_desc_force", "nn_pack", "nn_ens", "nn_decide", "k_fold32", "k_ljf"};
// statistics slots (unsigned long long)
enum { S_INCUT = 0, S_CIJ0 = 1, S_BSTAR = 2, S_DSB = 3, S_BONDS = 4, S_REBUILD = 5, S_MAXSHORT = 6, S_LJENT = 7,
       S_MAXLJ = 8, S_SPL = 9, S_SPL64 = 10, S_FALLBACK = 11, S_REGROW = 12, S_SLOW = 13, S_QUEUED = 14, S_INCUTF = 15,
       S_LFENT = 16, S_MAXLF = 17, S_N = 18 };

// One system of a batch: its own periodic box and cell grid.  A single
// configuration is a batch of one.
struct SysBox {
  double L[3], invL[3];
  int per[3];
  int nc[3];
  int cell_off;      // first cell of this system in the global cell arrays
  int natoms;
};

struct Dev {
  int n;
  int nsys;
  const SysBox* sys;       // [nsys]
  const int* atom_sys;     // [n] system of each atom (nullptr when nsys == 1)
  double* sys_acc;         // [nsys][A_N] per-system accumulators (nsys > 1)
  double skin, rlist2[3], rint2[3];
  double4* x;        // positions (w = species) since the last build
  double4* xref;     // positions at the last build
  float4* xsort;     // FP32 positions ordered by cell (list build only)
  int* cell_of;
  int* cell_count;
  int* cell_start;
  int* cell_cursor;
  int* cell_atoms;
  // LJ list in two parts, both full (every pair from both ends): near
  // pairs (within 3 max R2 + skin at the build, where C_ij < 1 and the S_r
  // range can occur) and far pairs (plain LJ for the list's lifetime)
  double rnear;      // near / far boundary at the build: 3 max R2 + skin
  int minimg;        // every periodic side >= 2 (LJ list cutoff + skin): far pairs by minimum image
  int lj_cap;
  int* lj_n;
  unsigned* lj_e;    // near: j | shift code << 27
  int lf_cap;
  int* lf_n;
  unsigned* lf_e;    // far: j | shift code << 27
  int icap;          // intermediate-list stride
  int* in_n;
  int* in_e;
  int scap, slog2;   // short-list stride (a power of two) and its log2
  int* sn;
  int* sj;
  double4* sd;       // displacement to neighbour and its length
  double2* sw;       // w, dw/dr
  double* NCt;
  double* NHt;
  int bcap;
  int* bcount;       // [3]
  int2* bonds;       // [3][bcap]: (i, slot)
  int qcap;          // capacity per queue segment
  int* qcount;       // [NSEG * QSTRIDE]
  int4* q;           // (i, j, shift code, path code)
  double* F;         // forces [n][3]
  float* F32;        // FP32 force sums [n][3], single precision only (folded into F, then cleared)
  double* acc;       // A_N accumulators
  unsigned long long* stats;
  int* flags;
  int* step;
  const int* skip;   // when set and nonzero, the force kernels return at once (surrogate step kept)
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sys_of(const Dev& D, int i) { return D.atom_sys ? D.atom_sys[i] : 0; }
__device__ __forceinline__ const SysBox& box_of(const Dev& D, int i) { return D.sys[sys_of(D, i)]; }
template <typename R> struct V3 { R x, y, z; };
template <typename R> __device__ __forceinline__ V3<R> mk(R a, R b, R c) { return {a, b, c}; }
template <typename R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename R> __device__ __forceinline__ V3<R> operator-(V3<R> a) { return {-a.x, -a.y, -a.z}; }
template <typename R> __device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename R> __device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ double xsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float xsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double xexp(double a) { return exp(a); }
__device__ __forceinline__ float xexp(float a) { return expf(a); }
__device__ __forceinline__ void xsincospi(double a, double* s, double* c) { sincospi(a, s, c); }
__device__ __forceinline__ void xsincospi(float a, float* s, float* c) { sincospif(a, s, c); }

// FP64 reciprocal and reciprocal square root: the hardware estimate refined
// by one Newton-Raphson step, which doubles its correct bits; the result is
// within a few ulp of the correctly rounded value at a fraction of the cost
// (and of the dependent latency) of the IEEE division and square root
// sequences.  FP32 keeps the compiler's operations.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);   // y <- y (1 + e / 2), e = 1 - x y^2
  return fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rcp_nr(float x) { return 1.0f / x; }
__device__ __forceinline__ float rsq_nr(float x) { return 1.0f / sqrtf(x); }

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// REBO bond weight w(r) and dw/dr: 1 below R1, 0 above R2, half cosine between.
template <typename R>
__device__ __forceinline__ R cutw(const DevParams& P, int p, R r, R& dw) {
  if (r <= (R)P.R1[p]) { dw = 0; return 1; }
  if (r >= (R)P.R2[p]) { dw = 0; return 0; }
  R t = (r - (R)P.R1[p]) * (R)P.inv_dR[p];
  R s, c;
  xsincospi(t, &s, &c);
  dw = (R)(-0.5 * M_PI) * (R)P.inv_dR[p] * s;
  return (R)0.5 * ((R)1 + c);
}
// Cubic switch S(t) = 1 - t^2 (3 - 2t) on [0,1] and dS/dt.
template <typename R>
__device__ __forceinline__ R Sw(R t, R& d) {
  if (t <= (R)0) { d = 0; return 1; }
  if (t >= (R)1) { d = 0; return 0; }
  d = (R)-6 * t * ((R)1 - t);
  return (R)1 - t * t * ((R)3 - (R)2 * t);
}
// Half-cosine step from 1 (x <= lo) to 0 (x >= hi).
template <typename R>
__device__ __forceinline__ R cosstep(R x, double lo, double hi, R& d) {
  if (x <= (R)lo) { d = 0; return 1; }
  if (x >= (R)hi) { d = 0; return 0; }
  R inv = (R)(1.0 / (hi - lo));
  R s, c;
  xsincospi((x - (R)lo) * inv, &s, &c);
  d = (R)(-0.5 * M_PI) * inv * s;
  return (R)0.5 * ((R)1 + c);
}
// Collinearity guard of dihedral terms as a function of cos theta.
template <typename R>
__device__ __forceinline__ R guard(const DevParams& P, R c, R& d) {
  R a = c < (R)0 ? -c : c;
  R inv = (R)P.inv_guard;
  R ds;
  R s = Sw((a - (R)P.guard_on) * inv, ds);
  d = ds * inv * (c < (R)0 ? (R)-1 : (R)1);
  return s;
}

// Quintic angular spline: value and d/dx.
template <typename R>
__device__ __forceinline__ R gspl(const GSpline& g, R x, R& d, int* st, double kd) {
  st[0]++;
  if constexpr (std::is_same<R, float>::value) {
    for (int m = 1; m + 1 < g.n; ++m)
      if (fabs((double)x - g.x[m]) < kd) {
        st[1]++;
        double dd;
        double v = gspl<double>(g, (double)x, dd, st + 2, kd);
        d = (float)dd;
        return (float)v;
      }
  }
  bool clamped = false;
  if (x <= (R)g.x[0]) { x = (R)g.x[0]; clamped = true; }
  if (x >= (R)g.x[g.n - 1]) { x = (R)g.x[g.n - 1]; clamped = true; }
  int m = 0;
  while (m + 2 < g.n && x > (R)g.x[m + 1]) ++m;
  R t = (x - (R)g.x[m]) * (R)g.inv_h[m];
  const double* c = g.c[m];
  R v = (R)c[5], dv = (R)0;
  for (int p = 4; p >= 0; --p) { dv = dv * t + v; v = v * t + (R)c[p]; }
  d = clamped ? (R)0 : dv * (R)g.inv_h[m];
  return v;
}
// g_i(cos theta) of the centre species; carbon blends gamma_C in over N_ij.
template <typename R>
__device__ __forceinline__ R gfun(const DevParams& P, int sc, R c, R N, R& dc, R& dN, int* st) {
  dN = 0;
  if (sc == 1) return gspl(P.gH, c, dc, st, P.knot_delta);
  R dG;
  R G = gspl(P.gC, c, dG, st, P.knot_delta);
  dc = dG;
  if (c <= (R)P.gammaC.x[0]) return G;
  R dQ;
  R Qn = cosstep(N, P.gC_lo, P.gC_hi, dQ);
  if (Qn == (R)0 && dQ == (R)0) return G;
  R dgam;
  R gam = gspl(P.gammaC, c, dgam, st, P.knot_delta);
  dc = dG + Qn * (dgam - dG);
  dN = dQ * (gam - G);
  return G + Qn * (gam - G);
}
// The same quintic spline in FP64 without branches (clamped argument,
// interval found by counting the interior knots below it: the knots
// increase), so that several evaluations can run as independent chains.
__device__ __forceinline__ double gspl_nb(const GSpline& g, double x, double& d) {
  const double x0 = g.x[0], xn = g.x[g.n - 1];
  const bool clamped = x <= x0 || x >= xn;
  x = fmin(fmax(x, x0), xn);
  int m = 0;
#pragma unroll
  for (int k = 1; k + 1 < kMaxKnots; ++k) m += (k + 1 < g.n && x > g.x[k]) ? 1 : 0;
  const double t = (x - g.x[m]) * g.inv_h[m];
  const double* c = g.c[m];
  double v = c[5], dv = 0.0;
  for (int q = 4; q >= 0; --q) { dv = dv * t + v; v = v * t + c[q]; }
  d = clamped ? 0.0 : dv * g.inv_h[m];
  return v;
}
// g_i(cos theta) as gfun, FP64, without branches; Qn, dQ: the blend weight
// of the centre's coordination (cosstep of N over [gC_lo, gC_hi]).
__device__ __forceinline__ double gfun_nb(const DevParams& P, int sc, double c, double Qn, double dQ, double& dc,
                                          double& dN, int* st) {
  double dG;
  const double G = gspl_nb(sc == 1 ? P.gH : P.gC, c, dG);
  double dgam;
  const double gam = gspl_nb(P.gammaC, c, dgam);
  const bool blend = sc == 0 && c > P.gammaC.x[0] && !(Qn == 0.0 && dQ == 0.0);
  st[0] += blend ? 2 : 1;
  dc = blend ? dG + Qn * (dgam - dG) : dG;
  dN = blend ? dQ * (gam - G) : 0.0;
  return blend ? G + Qn * (gam - G) : G;
}

// Bicubic P_{C s_j}(N^C, N^H) with partials.
template <typename R>
__device__ __forceinline__ R bicubic(const double (*Pc)[4][16], R x, R y, R& dx, R& dy, int* st, double kd) {
  st[0]++;
  if constexpr (std::is_same<R, float>::value) {
    if (fabs((double)x - rint((double)x)) < kd || fabs((double)y - rint((double)y)) < kd) {
      st[1]++;
      double ddx, ddy;
      double v = bicubic<double>(Pc, (double)x, (double)y, ddx, ddy, st + 2, kd);
      dx = (float)ddx;
      dy = (float)ddy;
      return (float)v;
    }
  }
  bool kx = x < (R)0 || x > (R)4, ky = y < (R)0 || y > (R)4;
  // clamped to the table (a NaN argument maps to the first cell)
  x = fmin(fmax(x, (R)0), (R)4);
  y = fmin(fmax(y, (R)0), (R)4);
  int cx = min((int)x, 3), cy = min((int)y, 3);
  R tx = x - (R)cx, ty = y - (R)cy;
  const double* c = Pc[cx][cy];
  R v = 0, vx = 0, vy = 0;
  for (int a = 3; a >= 0; --a) {
    R b0 = (R)c[a * 4 + 3], b1 = 0;
    for (int b = 2; b >= 0; --b) { b1 = b1 * ty + b0; b0 = b0 * ty + (R)c[a * 4 + b]; }
    vx = vx * tx + v;
    v = v * tx + b0;
    vy = vy * tx + b1;
  }
  dx = kx ? (R)0 : vx;
  dy = ky ? (R)0 : vy;
  return v;
}
// Tricubic table t at (x, y, z) with partials.
template <typename R>
__device__ __forceinline__ R tricubic(const DevParams& P, int t, R x, R y, R z, R& dx, R& dy, R& dz, int* st) {
  st[0]++;
  if constexpr (std::is_same<R, float>::value) {
    const double kd = P.knot_delta;
    if (fabs((double)x - rint((double)x)) < kd || fabs((double)y - rint((double)y)) < kd ||
        fabs((double)z - rint((double)z)) < kd) {
      st[1]++;
      double ddx, ddy, ddz;
      double v = tricubic<double>(P, t, (double)x, (double)y, (double)z, ddx, ddy, ddz, st + 2);
      dx = (float)ddx;
      dy = (float)ddy;
      dz = (float)ddz;
      return (float)v;
    }
  }
  bool kx = x < (R)0 || x > (R)4, ky = y < (R)0 || y > (R)4, kz = z < (R)1 || z > (R)9;
  // clamped to the table (a NaN argument maps to the first cell)
  x = fmin(fmax(x, (R)0), (R)4);
  y = fmin(fmax(y, (R)0), (R)4);
  z = fmin(fmax(z, (R)1), (R)9);
  int cx = min((int)x, 3), cy = min((int)y, 3), cz = min((int)z - 1, 7);
  int cell = (cx * 4 + cy) * 8 + cz;
  dx = dy = dz = 0;
  if (!P.tri_nz[t][cell]) return 0;
  R tx = x - (R)cx, ty = y - (R)cy, tz = z - (R)(cz + 1);
  const double* c = P.tri + ((size_t)t * kTriCells + cell) * kTriCoef;
  R v = 0, vx = 0, vy = 0, vz = 0;
  for (int a = 3; a >= 0; --a) {
    R u = 0, uy = 0, uz = 0;
    for (int b = 3; b >= 0; --b) {
      const double* cc = c + (a * 4 + b) * 4;
      R w = (R)cc[3], wz = 0;
      for (int k = 2; k >= 0; --k) { wz = wz * tz + w; w = w * tz + (R)cc[k]; }
      uy = uy * ty + u;
      u = u * ty + w;
      uz = uz * ty + wz;
    }
    vx = vx * tx + v;
    v = v * tx + u;
    vy = vy * tx + uy;
    vz = vz * tx + uz;
  }
  dx = kx ? (R)0 : vx;
  dy = ky ? (R)0 : vy;
  dz = kz ? (R)0 : vz;
  return v;
}

// ---------------------------------------------------------------------------
// Force / virial accumulation of one lane in type A (FP64, or FP32 in single
// precision).  A gradient g = dE/dr_ab on the relative vector r_ab = x_b - x_a
// gives F_a += g, F_b -= g and W -= r_ab (x) g; the two atoms the lane owns are
// kept in registers.
// ---------------------------------------------------------------------------
template <typename A_>
struct AccT {
  using A = A_;
  int st[4];         // spline evaluations, of which in FP64 near a knot
  int i, j;
  A fi[3], fj[3];
  A W[6];
  A* F;
  __device__ void init(A* F_, int i_, int j_) {
    F = F_; i = i_; j = j_;
    st[0] = st[1] = st[2] = st[3] = 0;
    for (int c = 0; c < 3; ++c) fi[c] = fj[c] = 0;
    for (int c = 0; c < 6; ++c) W[c] = 0;
  }
  __device__ void force(int a, A gx, A gy, A gz) {
    if (a == i) { fi[0] += gx; fi[1] += gy; fi[2] += gz; }
    else if (a == j) { fj[0] += gx; fj[1] += gy; fj[2] += gz; }
    else { atomic_add(&F[3 * a], gx); atomic_add(&F[3 * a + 1], gy); atomic_add(&F[3 * a + 2], gz); }
  }
  template <typename R>
  __device__ void vec(int a, int b, V3<R> r, V3<R> g, A scale = 1) {
    A gx = scale * (A)g.x, gy = scale * (A)g.y, gz = scale * (A)g.z;
    force(a, gx, gy, gz);
    force(b, -gx, -gy, -gz);
    A rx = r.x, ry = r.y, rz = r.z;
    W[0] -= rx * gx; W[1] -= ry * gy; W[2] -= rz * gz;
    W[3] -= rx * gy; W[4] -= rx * gz; W[5] -= ry * gz;
  }
  __device__ void flush() {
    if (i >= 0) for (int c = 0; c < 3; ++c) if (fi[c] != 0) atomic_add(&F[3 * i + c], fi[c]);
    if (j >= 0) for (int c = 0; c < 3; ++c) if (fj[c] != 0) atomic_add(&F[3 * j + c], fj[c]);
  }
};

// Force array a kernel accumulates into: FP64, or the FP32 sums of single precision.
template <typename A> __device__ __forceinline__ A* fbuf(const Dev& D);
template <> __device__ __forceinline__ double* fbuf<double>(const Dev& D) { return D.F; }
template <> __device__ __forceinline__ float* fbuf<float>(const Dev& D) { return D.F32; }

// Copy the parameter block into LDS (all threads of the block take part).
// The bond-order code reads spline knots and coefficients at lane-dependent
// addresses in long dependent chains; from LDS each of those reads costs a
// fraction of an L2 round trip.
__device__ __forceinline__ void stage_params(DevParams& dst, const DevParams* __restrict__ src) {
  static_assert(sizeof(DevParams) % 8 == 0, "parameter block is copied in 8-byte words");
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(&dst);
  for (int k = threadIdx.x; k < (int)(sizeof(DevParams) / 8); k += blockDim.x) d[k] = s[k];
  __syncthreads();
}

// Block reduction of `nv` doubles per thread into global accumulators.
template <int NV>
__device__ void block_reduce_add(double (&v)[NV], double* out) {
  __shared__ double red[NV][4];
  int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  for (int q = 0; q < NV; ++q) {
    double s = v[q];
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[q][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0;
    int nw = (blockDim.x + WAVE - 1) / WAVE;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    if (s != 0) atomic_add(&out[(blockIdx.x & (NSLOT - 1)) * A_N + threadIdx.x], s);
  }
}

// Add a lane's contribution to its system's accumulators (batched mode only).
// Wave-uniform systems are reduced first (one atomic per quantity).
template <int NV>
__device__ void sys_add(const Dev& D, int sysid, const double (&v)[NV], int base, bool active) {
  if (D.nsys <= 1) return;
  int lane = threadIdx.x & (WAVE - 1);
  int s0 = __shfl(active ? sysid : -1, 0);
  unsigned long long act = __ballot(active);
  bool uniform = __all(!active || sysid == s0) && (act & 1ull);
  if (uniform) {
    for (int q = 0; q < NV; ++q) {
      double t = active ? v[q] : 0.0;
      for (int o = WAVE / 2; o > 0; o >>= 1) t += __shfl_xor(t, o);
      if (lane == 0 && t != 0) atomic_add(&D.sys_acc[(size_t)s0 * A_N + base + q], t);
    }
  } else if (active) {
    for (int q = 0; q < NV; ++q)
      if (v[q] != 0) atomic_add(&D.sys_acc[(size_t)sysid * A_N + base + q], v[q]);
  }
}

__device__ __forceinline__ unsigned long long lanes_below() {
  int lane = threadIdx.x & (WAVE - 1);
  return lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
}
// Wave-aggregated append: every lane with `want` reserves `cnt` slots of the
// counter; one atomic per wavefront.  Returns the lane's first slot.
__device__ __forceinline__ int wave_append(int* counter, bool want, int cnt) {
  int lane = threadIdx.x & (WAVE - 1);
  int v = want ? cnt : 0;
  int incl = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  int total = __shfl(incl, WAVE - 1);
  int base = 0;
  if (lane == WAVE - 1 && total) base = atomicAdd(counter, total);
  base = __shfl(base, WAVE - 1);
  return base + incl - v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

template <typename R>
__device__ __forceinline__ V3<R> nbr_vec(const Dev& D, int a, int q, R& r) {
  double4 d = D.sd[a * D.scap + q];
  r = (R)d.w;
  return {(R)d.x, (R)d.y, (R)d.z};
}

// ---------------------------------------------------------------------------
// Neighbourhood of one bond (or deferred pair) i-j staged in LDS.  The
// bond-order passes (both ends forward, the dihedral loops, both ends
// reverse, the torsion) visit the short lists of i and j several times; read
// from memory each visit costs two dependent round trips per neighbour
// (list entry, then the neighbour's species and N).  The stage issues all of
// them at once per bond, so that a lane's dependent chain holds two round
// trips instead of about a hundred.  The first NB neighbours of each end are
// staged (every atom of a hydrocarbon at ordinary conditions); further ones
// are read from memory.  Layout [slot][thread] (slot = end * NB + q), so
// that a wavefront's accesses are consecutive.
// ---------------------------------------------------------------------------
constexpr int NB = 4;
template <typename R> struct alignas(4 * sizeof(R)) Q4 { R x, y, z, w; };
template <typename R> struct alignas(2 * sizeof(R)) Q2 { R x, y; };

// Bytes of the stage per thread.
template <typename R>
constexpr int stage_bytes() { return 2 * NB * (int)(sizeof(Q4<R>) + sizeof(Q2<R>) + sizeof(R) + sizeof(int)); }

// One neighbour k of an end centre c: its index and species, r_ck and its
// length, w_ck and dw/dr, and N_k (all neighbours of k, weighted).
template <typename R>
struct Nb {
  int k, s;
  V3<R> d;
  R r, w, dw, nt;
};

template <typename R>
struct Stage {
  Q4<R>* d;    // r_ck, |r_ck|
  Q2<R>* w;    // w_ck, dw_ck/dr
  R* nt;       // N_k
  int* ks;     // 2 k + species of k
  int T, t;             // threads of the block, this thread
  int c0, c1, n0, n1;   // end centres i, j and their list lengths
  __device__ int len(int e) const { return e ? n1 : n0; }
  __device__ void init(unsigned char* base) {
    T = blockDim.x;
    t = threadIdx.x;
    d = reinterpret_cast<Q4<R>*>(base);
    w = reinterpret_cast<Q2<R>*>(d + 2 * NB * T);
    nt = reinterpret_cast<R*>(w + 2 * NB * T);
    ks = reinterpret_cast<int*>(nt + 2 * NB * T);
  }
  // Stage the lists of i and j.
  __device__ void fill(const Dev& D, int i, int j) {
    c0 = i; c1 = j;
    n0 = D.sn[i]; n1 = D.sn[j];
    int kk[2 * NB];
#pragma unroll
    for (int u = 0; u < 2 * NB; ++u) {
      const int e = u / NB, q = u % NB;
      kk[u] = -1;
      if (q < (e ? n1 : n0)) {
        const int idx = (e ? c1 : c0) * D.scap + q;
        kk[u] = D.sj[idx];
        const double4 a = D.sd[idx];
        const double2 b = D.sw[idx];
        d[u * T + t] = {(R)a.x, (R)a.y, (R)a.z, (R)a.w};
        w[u * T + t] = {(R)b.x, (R)b.y};
      }
    }
#pragma unroll
    for (int u = 0; u < 2 * NB; ++u) {
      const int k = kk[u];
      if (k >= 0) {
        ks[u * T + t] = 2 * k + __double2int_rn(D.x[k].w);
        nt[u * T + t] = (R)(D.NCt[k] + D.NHt[k]);
      }
    }
  }
  // Neighbour q of end e (0: i, 1: j).
  __device__ Nb<R> get(const Dev& D, int e, int q) const {
    Nb<R> b;
    if (q < NB) {
      const int u = (e * NB + q) * T + t;
      const Q4<R> a = d[u];
      const Q2<R> v = w[u];
      const int x = ks[u];
      b.k = x >> 1;
      b.s = x & 1;
      b.d = {a.x, a.y, a.z};
      b.r = a.w;
      b.w = v.x;
      b.dw = v.y;
      b.nt = nt[u];
    } else {
      const int idx = (e ? c1 : c0) * D.scap + q;
      b.k = D.sj[idx];
      const double4 a = D.sd[idx];
      const double2 v = D.sw[idx];
      b.s = __double2int_rn(D.x[b.k].w);
      b.d = {(R)a.x, (R)a.y, (R)a.z};
      b.r = (R)a.w;
      b.w = (R)v.x;
      b.dw = (R)v.y;
      b.nt = (R)(D.NCt[b.k] + D.NHt[b.k]);
    }
    return b;
  }
};

// ---------------------------------------------------------------------------
// Bond order b_ij (Sec. 2.1.3).  One end at a time: end e (0: i, 1: j),
// centre c with partner o along r_co.  With bstar, r_ij is replaced by R1_ij
// where a bond length i-j enters (the lambda exponent); directions are kept.
// ---------------------------------------------------------------------------
template <typename R>
struct EndF {
  R NC, NH, N, S, P, dPC, dPH, p, conj, SdN;
  // FP64: g, dg/dcos and dg/dN of the staged neighbours (slot q < NB),
  // evaluated together by gslots and reused by the reverse pass
  R g[NB], dgc[NB], dgN[NB];
};

// Coordination of end e without its partner o: N^C, N^H and N.
template <typename R, typename SGT>
__device__ void end_n(const Dev& D, const SGT& SG, int ee, int o, EndF<R>& e) {
  const int n = SG.len(ee);
  R NC = 0, NH = 0;
  for (int q = 0; q < n; ++q) {
    const Nb<R> b = SG.get(D, ee, q);
    if (b.k == o) continue;
    if (b.s == 0) NC += b.w; else NH += b.w;
  }
  e.NC = NC; e.NH = NH; e.N = NC + NH;
}

// The angular splines of every staged neighbour of both ends (FP64), as
// 2 NB independent chains; slots beyond an end's list are left at zero.
template <typename SGT>
__device__ void gslots(const DevParams& P, const Dev& D, const SGT& SG, int i, int j, int si, int sj, V3<double> rij,
                       double r, EndF<double>& ei, EndF<double>& ej, int* st) {
  const double ir = rcp_nr(r);
  double Q[2], dQ[2];
  Q[0] = cosstep(ei.N, P.gC_lo, P.gC_hi, dQ[0]);
  Q[1] = cosstep(ej.N, P.gC_lo, P.gC_hi, dQ[1]);
#pragma unroll
  for (int u = 0; u < 2 * NB; ++u) {
    const int e = u / NB, q = u % NB;
    EndF<double>& ef = e ? ej : ei;
    const Nb<double> b = SG.get(D, e, q);
    const bool valid = q < SG.len(e) && b.k != (e ? i : j);
    const double sgn = e ? -1.0 : 1.0;
    const double cth = sgn * dot(rij, b.d) * (ir * rcp_nr(b.r));
    double dc, dN;
    int stq[1] = {0};
    const double g = gfun_nb(P, e ? sj : si, cth, Q[e], dQ[e], dc, dN, stq);
    if (valid) st[0] += stq[0];
    ef.g[q] = valid ? g : 0.0;
    ef.dgc[q] = valid ? dc : 0.0;
    ef.dgN[q] = valid ? dN : 0.0;
  }
}

template <typename R>
__device__ void end_fwd(const DevParams& P, const Dev& D, const Stage<R>& SG, int ee, int sc, int o, int so, V3<R> rco,
                        R rlen, R rlam, EndF<R>& e, int* st) {
  // e.NC, e.NH, e.N from end_n; in FP64 the staged neighbours' splines from gslots
  const int n = SG.len(ee);
  const R NC = e.NC, NH = e.NH, N = e.N;
  R S = 0, conj = 0, SdN = 0;
  const R irlen = rcp_nr(rlen);
  auto term = [&](const Nb<R>& b, R g, R dgN) {
    const int sk = b.s;
    const R r = b.r, w = b.w;
    R el = 1;
    if (sc == 1) el = xexp((R)P.lambda_pref * (((R)P.rho[sk] - r) - ((R)P.rho[so] - rlam)));
    S += w * g * el;
    SdN += w * el * dgN;
    if (sk == 0) {
      R xk = b.nt - w;
      R dF;
      conj += w * cosstep(xk, P.conj_lo, P.conj_hi, dF);
    }
  };
  int q0 = 0;
  if constexpr (std::is_same<R, double>::value) {
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q < n) {
        const Nb<R> b = SG.get(D, ee, q);
        if (b.k != o) term(b, e.g[q], e.dgN[q]);
      }
    }
    q0 = NB;
  }
  for (int q = q0; q < n; ++q) {
    const Nb<R> b = SG.get(D, ee, q);
    if (b.k == o) continue;
    R cth = dot(rco, b.d) * (irlen * rcp_nr(b.r));
    R dgc, dgN;
    R g = gfun(P, sc, cth, N, dgc, dgN, st);
    term(b, g, dgN);
  }
  R Pv = 0, dPC = 0, dPH = 0;
  if (sc == 0) Pv = bicubic(P.Pc[so], NC, NH, dPC, dPH, st, P.knot_delta);
  e.S = S; e.P = Pv; e.dPC = dPC; e.dPH = dPH;
  e.p = rsq_nr((R)1 + S + Pv);
  e.conj = conj;
  e.SdN = SdN;
}

// Reverse pass of one end.  Gp = dE/dp, GN = dE/dN_co from outside the end,
// Gconj = dE/d(conjugation sum of this end).  Returns dE/dr_co in gco.
template <typename R, typename AC>
__device__ void end_rev(const DevParams& P, const Dev& D, const Stage<R>& SG, int ee, int c, int sc, int o, int so,
                        V3<R> rco, R rlen, R rlam, bool bstar, const EndF<R>& e, R Gp, R GN, R Gconj, V3<R>& gco,
                        AC& acc) {
  const int n = SG.len(ee);
  R GS = (R)-0.5 * e.p * e.p * e.p * Gp;
  R GNt = GN + GS * e.SdN;
  R GNC = GS * e.dPC + GNt, GNH = GS * e.dPH + GNt;
  R Grlen = 0;
  const R irlen = rcp_nr(rlen);
  auto term = [&](const Nb<R>& b, R g, R dgc) {
    const int k = b.k;
    const int sk = b.s;
    const R r = b.r, w = b.w, dw = b.dw;
    const V3<R> d = b.d;
    const R ir = rcp_nr(r);
    R inv = irlen * ir;
    R cth = dot(rco, d) * inv;
    R el = 1;
    R Gr = 0;
    if (sc == 1) {
      el = xexp((R)P.lambda_pref * (((R)P.rho[sk] - r) - ((R)P.rho[so] - rlam)));
      R Gl = GS * w * g * el * (R)P.lambda_pref;
      Gr -= Gl;
      if (!bstar) Grlen += Gl;
    }
    R Gw = GS * g * el + (sk == 0 ? GNC : GNH);
    R Gcos = GS * w * el * dgc;
    if (sk == 0) {
      R xk = b.nt - w;
      R dF;
      R Fv = cosstep(xk, P.conj_lo, P.conj_hi, dF);
      Gw += Gconj * Fv;
      R Gx = Gconj * w * dF;
      if (Gx != (R)0) {
        int nk = D.sn[k];
        for (int u = 0; u < nk; ++u) {
          int m = D.sj[k * D.scap + u];
          if (m == c) continue;
          R rm;
          V3<R> dm = nbr_vec<R>(D, k, u, rm);
          R dwm = (R)D.sw[k * D.scap + u].y;
          if (dwm != (R)0) acc.vec(k, m, dm, (Gx * dwm * rcp_nr(rm)) * dm);
        }
      }
    }
    Gr += Gw * dw;
    V3<R> gk = (Gr * ir) * d + Gcos * (inv * rco - (cth * ir * ir) * d);
    gco = gco + Gcos * (inv * d - (cth * irlen * irlen) * rco);
    acc.vec(c, k, d, gk);
  };
  int q0 = 0;
  if constexpr (std::is_same<R, double>::value) {   // the forward pass's slot splines
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q < n) {
        const Nb<R> b = SG.get(D, ee, q);
        if (b.k != o) term(b, e.g[q], e.dgc[q]);
      }
    }
    q0 = NB;
  }
  for (int q = q0; q < n; ++q) {
    const Nb<R> b = SG.get(D, ee, q);
    if (b.k == o) continue;
    R cth = dot(rco, b.d) * (irlen * rcp_nr(b.r));
    R dgc, dgN;
    R g = gfun(P, sc, cth, e.N, dgc, dgN, acc.st);
    term(b, g, dgc);
  }
  gco = gco + (Grlen * irlen) * rco;
}

// Dihedral loop over k in N(i)\{j}, l in N(j)\{i,k} of a C-C bond: forward
// sums of the pi^dh term (1 - cos^2) w_ik w_jl s_i s_j and of the torsion
// energy w_ik w_ij w_jl s_i s_j V(omega); with rev, the reverse pass given
// GSdh = dE/d(sum) and the torsion's own derivatives.
template <typename R, typename AC>
__device__ void dihedral(const DevParams& P, const Dev& D, const Stage<R>& SG, int i, int j, V3<R> rij, R r, R wij,
                         bool tors, bool rev, R GSdh, R& Sdh, R& Et, V3<R>& gij, R& Gwij, AC& acc) {
  const int ni = SG.n0, nj = SG.n1;
  V3<R> rji = -rij;
  const R ir = rcp_nr(r);
  for (int q = 0; q < ni; ++q) {
    const Nb<R> bk = SG.get(D, 0, q);
    const int k = bk.k;
    if (k == j) continue;
    const R rik_l = bk.r, wik = bk.w, dwik = bk.dw;
    const V3<R> rik = bk.d;
    const R irik = rcp_nr(rik_l);
    R ci = dot(rij, rik) * (ir * irik);
    R dgi;
    R gi = guard(P, ci, dgi);
    if (gi == (R)0) continue;
    V3<R> a = cross(rij, rik);
    R na2 = dot(a, a);
    const R ina = rsq_nr(na2);   // |a| > 0: the guard vanishes for collinear bonds
    const int sk = bk.s;
    V3<R> gik_sum = {0, 0, 0};   // dE/dr_ik summed over l (one force update per k)
    for (int u = 0; u < nj; ++u) {
      const Nb<R> bl = SG.get(D, 1, u);
      const int l = bl.k;
      if (l == i || l == k) continue;
      const R rjl_l = bl.r, wjl = bl.w, dwjl = bl.dw;
      const V3<R> rjl = bl.d;
      const R irjl = rcp_nr(rjl_l);
      R cj = dot(rji, rjl) * (ir * irjl);
      R dgj;
      R gj = guard(P, cj, dgj);
      if (gj == (R)0) continue;
      V3<R> b = cross(rij, rjl);
      R nb2 = dot(b, b);
      const R inb = rsq_nr(nb2);
      R inab = ina * inb;
      R cw = dot(a, b) * inab;
      R ww = wik * wjl * gi * gj;
      Sdh += ((R)1 - cw * cw) * ww;
      R V = 0, dV = 0;
      if (tors) {
        R eps = (R)P.tors_eps[sk + bl.s];
        R h = (R)0.5 * ((R)1 + cw);
        R h2 = h * h, h4 = h2 * h2;
        V = eps * ((R)(256.0 / 405.0) * h4 * h - (R)0.1);
        dV = eps * (R)(256.0 / 405.0 * 2.5) * h4;
        Et += wij * ww * V;
      }
      if (!rev) continue;
      R Gc = GSdh * (R)-2 * cw * ww + wij * ww * dV;
      R Gww = GSdh * ((R)1 - cw * cw) + wij * V;
      Gwij += ww * V;
      R Gwik = Gww * wjl * gi * gj, Gwjl = Gww * wik * gi * gj;
      R Gci = Gww * wik * wjl * gj * dgi, Gcj = Gww * wik * wjl * gi * dgj;
      V3<R> Ga = Gc * (inab * b - (cw * ina * ina) * a);
      V3<R> Gb = Gc * (inab * a - (cw * inb * inb) * b);
      R iik = ir * irik, ijl = ir * irjl;
      V3<R> gik = cross(Ga, rij) + (Gwik * dwik * irik) * rik + Gci * (iik * rij - (ci * irik * irik) * rik);
      V3<R> gjl = cross(Gb, rij) + (Gwjl * dwjl * irjl) * rjl + Gcj * (ijl * rji - (cj * irjl * irjl) * rjl);
      gij = gij + cross(rik, Ga) + cross(rjl, Gb) + Gci * (iik * rik - (ci * ir * ir) * rij);
      gij = gij - Gcj * (ijl * rjl - (cj * ir * ir) * rji);
      gik_sum = gik_sum + gik;
      acc.vec(j, l, rjl, gjl);
    }
    if (rev) acc.vec(i, k, rik, gik_sum);
  }
}

// Forward state of one bond order, kept for its reverse pass.
template <typename R>
struct BondFwd {
  EndF<R> ei, ej;
  R rlam, Fij, Fji, dFc, Tv, dTa, dTb, dTc, Sdh;
  int si, sj;
  bool dh;
};

// Bond order b_ij, forward pass only; fills the state of the reverse pass.
template <typename R>
__device__ R bond_order_fwd(const DevParams& P, const Dev& D, const Stage<R>& SG, int i, int j, V3<R> rij, R r,
                            bool bstar, BondFwd<R>& f, int* st) {
  int si = __double2int_rn(D.x[i].w), sj = __double2int_rn(D.x[j].w);
  int p = si + sj;
  f.si = si; f.sj = sj;
  f.rlam = (bstar && P.bstar_use_R1) ? (R)P.R1[p] : r;
  V3<R> rji = -rij;
  end_n(D, SG, 0, j, f.ei);
  end_n(D, SG, 1, i, f.ej);
  if constexpr (std::is_same<R, double>::value) gslots(P, D, SG, i, j, si, sj, rij, r, f.ei, f.ej, st);
  end_fwd(P, D, SG, 0, si, j, sj, rij, r, f.rlam, f.ei, st);
  end_fwd(P, D, SG, 1, sj, i, si, rji, r, f.rlam, f.ej, st);
  R Nconj = (R)1 + f.ei.conj * f.ei.conj + f.ej.conj * f.ej.conj;
  R dFa, dFb;
  R pirc;
  bool swap = (p == 1 && si == 1);   // C-H table takes the carbon side first
  int tF = p == 0 ? TRI_FCC : (p == 1 ? TRI_FCH : TRI_FHH);
  if (!swap) { pirc = tricubic(P, tF, f.ei.N, f.ej.N, Nconj, dFa, dFb, f.dFc, st); f.Fij = dFa; f.Fji = dFb; }
  else { pirc = tricubic(P, tF, f.ej.N, f.ei.N, Nconj, dFa, dFb, f.dFc, st); f.Fij = dFb; f.Fji = dFa; }
  f.Tv = 0; f.dTa = 0; f.dTb = 0; f.dTc = 0; f.Sdh = 0;
  f.dh = false;
  if (p == 0) {
    f.Tv = tricubic(P, TRI_TCC, f.ei.N, f.ej.N, Nconj, f.dTa, f.dTb, f.dTc, st);
    f.dh = f.Tv != (R)0 || f.dTa != (R)0 || f.dTb != (R)0 || f.dTc != (R)0;
    if (f.dh) {
      V3<R> dummy = {0, 0, 0};
      R Et = 0, Gwij = 0;
      AccT<double> none;   // forward only: nothing is accumulated
      none.st[0] = none.st[1] = 0;
      dihedral(P, D, SG, i, j, rij, r, (R)0, false, false, (R)0, f.Sdh, Et, dummy, Gwij, none);
    }
  }
  return (R)0.5 * (f.ei.p + f.ej.p) + pirc + f.Tv * f.Sdh;
}

// Reverse pass of a bond order for dE/db = Gb, from its forward state.
// With dihedral_done, the caller takes the pi^dh part of the dihedral loop
// (dE/dSdh = Gb T_ij) together with its own pass over the same loop.
template <typename R, typename AC>
__device__ void bond_order_rev(const DevParams& P, const Dev& D, const Stage<R>& SG, int i, int j, V3<R> rij, R r,
                               bool bstar, const BondFwd<R>& f, R Gb, V3<R>& gij, AC& acc,
                               bool dihedral_done = false) {
  R GNij = Gb * (f.Fij + f.Sdh * f.dTa), GNji = Gb * (f.Fji + f.Sdh * f.dTb), GNc = Gb * (f.dFc + f.Sdh * f.dTc);
  if (f.dh && !dihedral_done) {
    R s2 = 0, Et = 0, Gwij = 0;
    dihedral(P, D, SG, i, j, rij, r, (R)0, false, true, Gb * f.Tv, s2, Et, gij, Gwij, acc);
  }
  V3<R> gi = {0, 0, 0}, gj = {0, 0, 0};
  V3<R> rji = -rij;
  end_rev(P, D, SG, 0, i, f.si, j, f.sj, rij, r, f.rlam, bstar, f.ei, (R)0.5 * Gb, GNij, GNc * (R)2 * f.ei.conj, gi,
          acc);
  end_rev(P, D, SG, 1, j, f.sj, i, f.si, rji, r, f.rlam, bstar, f.ej, (R)0.5 * Gb, GNji, GNc * (R)2 * f.ej.conj, gj,
          acc);
  gij = gij + gi - gj;
}

// ---------------------------------------------------------------------------
// Kernels: neighbour lists
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_coord(double x, double invL, int nc) {
  int c = (int)floor(x * invL * nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Load positions (wrapping periodic dims), reset cell counters.
__global__ void k_load(Dev D, const double* __restrict__ pos, const int* __restrict__ spec, int wrap_only) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  double4 x;
  if (wrap_only) {
    x = D.x[i];
  } else {
    x = make_double4(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], (double)spec[i]);
    if (spec[i] != 0 && spec[i] != 1) atomicOr(D.flags, F_BADSPEC);
  }
  double* xc = &x.x;
  const SysBox& B = box_of(D, i);
  for (int c = 0; c < 3; ++c) {
    if (!isfinite(xc[c])) atomicOr(D.flags, F_NONFINITE);
    if (B.per[c]) {
      xc[c] -= B.L[c] * floor(xc[c] * B.invL[c]);
      if (xc[c] >= B.L[c]) xc[c] -= B.L[c];
      if (xc[c] < 0) xc[c] = 0;
    }
  }
  D.x[i] = x;
}

// Counters of the last-block patterns (D.step[1], D.step[2]): every block
// of a kernel adds one after its own work; the block that brings the count
// to gridDim.x finishes the kernel's sequential tail and resets the count.
// Each thread's writes are released at device scope before the block's
// barrier and the counter update, and acquired again by the last block, so
// the tail sees every block's atomics (the usual threadfence reduction).
__device__ __forceinline__ bool last_block(int* counter) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0)
    is_last = __hip_atomic_fetch_add(counter, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (int)gridDim.x - 1;
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  return true;
}

// Binning of a rebuild (wrapped positions, reference positions, cell of
// every atom, cell counts); the last block to finish turns the counts into
// cell starts (exclusive scan) and clears them for the next build.
__global__ void k_bin(Dev D, int ncell) {
  if (!(*D.flags & F_REBUILD)) return;   // the same on every block
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < D.n) {
    double4 x = D.x[i];
    double* xc = &x.x;
    const SysBox& B = box_of(D, i);
    for (int c = 0; c < 3; ++c) {
      if (B.per[c]) {
        xc[c] -= B.L[c] * floor(xc[c] * B.invL[c]);
        if (xc[c] >= B.L[c]) xc[c] -= B.L[c];
        if (xc[c] < 0) xc[c] = 0;
      }
    }
    D.x[i] = x;
    D.xref[i] = x;
    int c = B.cell_off + (cell_coord(x.x, B.invL[0], B.nc[0]) * B.nc[1] + cell_coord(x.y, B.invL[1], B.nc[1])) * B.nc[2] +
            cell_coord(x.z, B.invL[2], B.nc[2]);
    D.cell_of[i] = c;
    atomicAdd(&D.cell_count[c], 1);
  }
  if (!last_block(D.step + 2)) return;
  // block-wide exclusive scan of the per-thread sums: within each wavefront
  // by shuffles, then over the wavefront totals
  __shared__ int wtot[1024 / WAVE];
  int t = threadIdx.x, nt = blockDim.x;
  int per = (ncell + nt - 1) / nt;
  int lo = t * per, hi = min(ncell, lo + per);
  int sum = 0;
  for (int c = lo; c < hi; ++c) sum += D.cell_count[c];
  const int lane = t & (WAVE - 1), w = t / WAVE;
  int incl = sum;
  for (int o = 1; o < WAVE; o <<= 1) {
    int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == WAVE - 1) wtot[w] = incl;
  __syncthreads();
  int wbase = 0;
  for (int q = 0; q < w; ++q) wbase += wtot[q];
  int run = wbase + incl - sum;
  for (int c = lo; c < hi; ++c) {
    D.cell_start[c] = run;
    D.cell_cursor[c] = run;
    run += D.cell_count[c];
    D.cell_count[c] = 0;
  }
  if (t == 0) {
    D.cell_start[ncell] = D.n;
    D.step[2] = 0;
  }
}

__global__ void k_fill(Dev D) {
  if (!(*D.flags & F_REBUILD)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  int slot = atomicAdd(&D.cell_cursor[D.cell_of[i]], 1);
  D.cell_atoms[slot] = i;
  double4 x = D.x[i];
  D.xsort[slot] = make_float4((float)x.x, (float)x.y, (float)x.z, (float)x.w);
}

// One wavefront per atom: full LJ list (cutoff + skin, with image shift code)
// and intermediate REBO list (R2 + skin), compacted with wave ballots.
// Cells are at least half the list cutoff, so the 5 x 5 x 5 cells around
// the atom's own hold every candidate.  Their candidates form one stream
// (each lane finds its cell by a binary search over the per-cell prefix
// counts in LDS); the atom index and FP32 position of the next block of 64
// candidates are loaded while this block is tested.  The FP32 test uses
// cutoffs enlarged by 1e-3 A, far above its rounding error (~1e-4 A at 500 A
// coordinates), so both lists contain every pair within the exact cutoffs;
// every consumer tests distances again in FP64.
constexpr int NSTEN = 125;   // cells of the stencil
__global__ __launch_bounds__(256) void k_build(Dev D, const DevParams* __restrict__ Pp) {
  if (!(*D.flags & F_REBUILD)) return;
  __shared__ int s_pre[4][NSTEN + 1];       // first stream index of each cell (last: total)
  __shared__ int s_start[4][NSTEN];         // first slot of the cell in the cell-ordered arrays
  __shared__ unsigned s_code[4][NSTEN];     // image shift code of the cell
  int lane = threadIdx.x & (WAVE - 1);
  int wv = threadIdx.x / WAVE;
  // one atom per wavefront (wave-uniform index: the atom's data in scalar registers)
  int i = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
  if (i >= D.n) return;
  double4 xi = D.x[i];
  int si = __double2int_rn(xi.w);
  const SysBox& B = box_of(D, i);
  int ci[3] = {cell_coord(xi.x, B.invL[0], B.nc[0]), cell_coord(xi.y, B.invL[1], B.nc[1]),
               cell_coord(xi.z, B.invL[2], B.nc[2])};
  // Cells whose box lies farther from the atom than the list cutoff (plus a
  // margin far above rounding) hold no candidate and are dropped: about 40%
  // of the stencil.  A wrapped atom lies in its cell's box; on a
  // non-periodic axis the edge cells also hold the atoms beyond the box
  // (cell_coord clamps), so they are unbounded outward.
  const double xa[3] = {xi.x, xi.y, xi.z};
  double hc[3];
  for (int c = 0; c < 3; ++c) hc[c] = B.L[c] / B.nc[c];
  const double rcut = sqrt(fmax(D.rlist2[0], fmax(D.rlist2[1], D.rlist2[2]))) + 0.01;
  int run = 0;   // candidates of the cells before this group of 64
  for (int o0 = 0; o0 < NSTEN; o0 += WAVE) {
    int o = o0 + lane;
    int cnt = 0, start = 0;
    unsigned code = 13;
    if (o < NSTEN) {
      int off[3] = {o / 25 - 2, (o / 5) % 5 - 2, o % 5 - 2};
      int cc[3], sh[3];
      bool skip = false;
      for (int c = 0; c < 3; ++c) {
        int u = ci[c] + off[c];
        if (B.per[c]) {
          sh[c] = u < 0 ? -1 : (u >= B.nc[c] ? 1 : 0);
          cc[c] = u - sh[c] * B.nc[c];
          if (cc[c] < 0 || cc[c] >= B.nc[c]) skip = true;   // small grids wrap once only
        } else {
          sh[c] = 0;
          cc[c] = u;
          if (u < 0 || u >= B.nc[c]) skip = true;
        }
      }
      code = (unsigned)((sh[0] + 1) * 9 + (sh[1] + 1) * 3 + (sh[2] + 1));
      double g2 = 0.0;   // squared distance from the atom to the cell's box (image frame)
      for (int c = 0; c < 3; ++c) {
        int u = ci[c] + off[c];
        double lo = u * hc[c], hi = lo + hc[c];
        if (!B.per[c] && u == 0) lo = -INFINITY;
        if (!B.per[c] && u == B.nc[c] - 1) hi = INFINITY;
        double g = fmax(0.0, fmax(lo - xa[c], xa[c] - hi));
        g2 += g * g;
      }
      if (g2 > rcut * rcut) skip = true;
      if (!skip) {
        int cell = B.cell_off + (cc[0] * B.nc[1] + cc[1]) * B.nc[2] + cc[2];
        start = D.cell_start[cell];
        cnt = D.cell_start[cell + 1] - start;
      }
    }
    int incl = cnt;
    for (int q = 1; q < WAVE; q <<= 1) {
      int u = __shfl_up(incl, q);
      if (lane >= q) incl += u;
    }
    if (o < NSTEN) { s_pre[wv][o] = run + incl - cnt; s_start[wv][o] = start; s_code[wv][o] = code; }
    run += __shfl(incl, WAVE - 1);
  }
  if (lane == 0) s_pre[wv][NSTEN] = run;
  int total = run;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // stream position v -> slot in the cell-ordered arrays and shift code
  auto locate = [&](int v, int& slot, unsigned& cd) {
    int lo = 0, hi = NSTEN;   // s_pre[lo] <= v < s_pre[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (s_pre[wv][mid] <= v) lo = mid; else hi = mid;
    }
    slot = s_start[wv][lo] + (v - s_pre[wv][lo]);
    cd = s_code[wv][lo];
  };
  float rlf[3], rif[3];
  for (int p = 0; p < 3; ++p) {
    float a = (float)sqrt(D.rlist2[p]) + 1e-3f, b = (float)sqrt(D.rint2[p]) + 1e-3f;
    rlf[p] = a * a;
    rif[p] = b * b;
  }
  // a pair goes to the far part only if its FP32 distance is beyond the
  // boundary by more than the FP32 rounding, so every pair that can come
  // within 3 max R2 before the next build is in the near part
  const float rnf = ((float)D.rnear + 1e-3f) * ((float)D.rnear + 1e-3f);
  float xix = (float)xi.x, xiy = (float)xi.y, xiz = (float)xi.z;
  float Lx = (float)B.L[0], Ly = (float)B.L[1], Lz = (float)B.L[2];
  int nlj = 0, nlf = 0, nin = 0;
  unsigned long long below = lanes_below();
  int j_n = -1;
  float4 x_n = make_float4(0.f, 0.f, 0.f, 0.f);
  unsigned c_n = 13;
  if (lane < total) {
    int slot;
    locate(lane, slot, c_n);
    j_n = D.cell_atoms[slot];
    x_n = D.xsort[slot];
  }
  for (int base = 0; base < total; base += WAVE) {
    int v = base + lane;
    int j = j_n;
    float4 xj = x_n;
    unsigned cd = c_n;
    if (v + WAVE < total) {
      int slot;
      locate(v + WAVE, slot, c_n);
      j_n = D.cell_atoms[slot];
      x_n = D.xsort[slot];
    }
    bool ok_lj = false, ok_in = false, far = false;
    if (v < total) {
      float dx = xj.x + (float)((int)(cd / 9) - 1) * Lx - xix;
      float dy = xj.y + (float)((int)((cd / 3) % 3) - 1) * Ly - xiy;
      float dz = xj.z + (float)((int)(cd % 3) - 1) * Lz - xiz;
      float r2 = dx * dx + dy * dy + dz * dz;
      int p = si + (xj.w != 0.0f ? 1 : 0);
      float rl = p == 0 ? rlf[0] : (p == 1 ? rlf[1] : rlf[2]);
      float ri = p == 0 ? rif[0] : (p == 1 ? rif[1] : rif[2]);
      bool self = (j == i) && cd == 13;
      ok_lj = !self && r2 < rl;
      ok_in = !self && r2 < ri;
      far = r2 >= rnf;
    }
    unsigned long long m = __ballot(ok_lj && !far);
    if (ok_lj && !far) {
      int pos = nlj + __popcll(m & below);
      if (pos < D.lj_cap) D.lj_e[(size_t)i * D.lj_cap + pos] = (unsigned)j | (cd << 27);
    }
    nlj += __popcll(m);
    m = __ballot(ok_lj && far);
    if (ok_lj && far) {
      int pos = nlf + __popcll(m & below);
      if (pos < D.lf_cap) D.lf_e[(size_t)i * D.lf_cap + pos] = (unsigned)j | (cd << 27);
    }
    nlf += __popcll(m);
    m = __ballot(ok_in);
    if (ok_in) {
      int pos = nin + __popcll(m & below);
      if (pos < D.icap) D.in_e[(size_t)i * D.icap + pos] = j;
    }
    nin += __popcll(m);
  }
  if (lane == 0) {
    D.lj_n[i] = nlj;            // unclamped; readers clamp to lj_cap / lf_cap
    D.lf_n[i] = nlf;
    D.in_n[i] = min(nin, D.icap);
    if (nlj > D.lj_cap || nlf > D.lf_cap) atomicOr(D.flags, F_OV_LJ);
    if (nin > D.icap) atomicOr(D.flags, F_OV_INT);
  }
}

// ---------------------------------------------------------------------------
// Kernels: per-step force evaluation
// ---------------------------------------------------------------------------
__global__ void k_zero(Dev D) {
  if (D.skip && *D.skip) return;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = t; k < 3 * D.n; k += gridDim.x * blockDim.x) D.F[k] = 0;
  if (D.F32)
    for (int k = t; k < 3 * D.n; k += gridDim.x * blockDim.x) D.F32[k] = 0;
  if (t < NSLOT * A_N) D.acc[t] = 0;
  if (D.nsys > 1)
    for (int k = t; k < D.nsys * A_N; k += gridDim.x * blockDim.x) D.sys_acc[k] = 0;
  if (t < 3) D.bcount[t] = 0;
  if (t < NSEG) D.qcount[t * QSTRIDE] = 0;
}

// Single precision: add the FP32 force sums into the FP64 forces the
// integrator and the caller read, and clear them for the next evaluation.
__global__ void k_fold32(Dev D) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < 3 * D.n; k += gridDim.x * blockDim.x) {
    float f = D.F32[k];
    D.F32[k] = 0.0f;
    D.F[k] += (double)f;
  }
}

__device__ __forceinline__ double xrint(double a) { return rint(a); }
__device__ __forceinline__ float xrint(float a) { return rintf(a); }
template <typename T>
__device__ __forceinline__ void minimg(const SysBox& B, T& dx, T& dy, T& dz) {
  if (B.per[0]) dx -= (T)B.L[0] * xrint(dx * (T)B.invL[0]);
  if (B.per[1]) dy -= (T)B.L[1] * xrint(dy * (T)B.invL[1]);
  if (B.per[2]) dz -= (T)B.L[2] * xrint(dz * (T)B.invL[2]);
}

// Exact short list, weights and coordination; species-bucketed bond list.
// S (single precision): relative vectors from FP32 positions, lengths,
// weights and coordination sums in FP32.
template <bool S>
__global__ __launch_bounds__(1024) void k_short(Dev D, const DevParams* __restrict__ Pp) {
  using T = typename std::conditional<S, float, double>::type;
  // the lists of this step's rebuild (if any) are complete: count it and
  // clear the flag (the list kernels are the only ones that read it)
  if (blockIdx.x == 0 && threadIdx.x == 0 && (*D.flags & F_REBUILD)) {
    atomicAnd(D.flags, ~F_REBUILD);
    D.stats[S_REBUILD] += 1;
  }
  if (D.skip && *D.skip) return;
  const DevParams& P = *Pp;
  // SG lanes per atom: lane `sub` of the group takes intermediate entries
  // sub, sub + SG, ...; the valid ones are compacted in entry order
  constexpr int SG = SHORT_G;
  static_assert(WAVE % SG == 0 && SCAP_MAX % SG == 0, "short-list groups");
  // pair class of each short neighbour j > i of the block's atoms (-1: j < i),
  // read back by slot for the bond list
  __shared__ signed char s_cls[1024 / SG][SCAP_MAX];
  int lane = threadIdx.x & (WAVE - 1);
  int sub = lane & (SG - 1);
  int la = threadIdx.x / SG;
  unsigned long long gmask = ((1ull << SG) - 1) << (lane & ~(SG - 1));
  unsigned long long below = lanes_below();
  const int scap = D.scap, icap = D.icap;
  int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / SG);
  bool live = i < D.n;
  double4 xi = make_double4(0, 0, 0, 0);
  int si = 0, m = 0;
  if (live) {
    xi = D.x[i];
    si = __double2int_rn(xi.w);
    m = D.in_n[i];
  }
  const SysBox& B = box_of(D, live ? i : 0);
  int mmax = wave_max(m);
  int cnt = 0;                // valid entries of atom i so far (uniform in the group)
  T NC = 0, NH = 0;           // partial sums of this lane
  for (int k = 0; k * SG < mmax; ++k) {   // wave-uniform trip count
    int e = k * SG + sub;
    bool ok = false;
    int j = 0, p = 0;
    double dx = 0, dy = 0, dz = 0, r = 0, w = 0, dw = 0;
    if (live && e < m) {
      j = D.in_e[(size_t)i * icap + e];
      double4 xj = D.x[j];
      T tx = (T)xj.x - (T)xi.x, ty = (T)xj.y - (T)xi.y, tz = (T)xj.z - (T)xi.z;
      minimg(B, tx, ty, tz);
      T r2 = tx * tx + ty * ty + tz * tz;
      int sj = __double2int_rn(xj.w);
      p = si + sj;
      if (r2 < P.R2[p] * P.R2[p]) {
        ok = true;
        T rt = xsqrt(r2), dwt;
        T wt = cutw<T>(P, p, rt, dwt);
        dx = tx; dy = ty; dz = tz; r = rt; w = wt; dw = dwt;
        if (sj == 0) NC += wt; else NH += wt;
      }
    }
    unsigned long long bal = __ballot(ok) & gmask;
    if (ok) {
      int pos = cnt + __popcll(bal & below);
      if (pos < scap) {
        D.sj[i * scap + pos] = j;
        D.sd[i * scap + pos] = make_double4(dx, dy, dz, r);
        D.sw[i * scap + pos] = make_double2(w, dw);
        s_cls[la][pos] = (signed char)(j > i ? p : -1);
      }
    }
    cnt += __popcll(bal);
  }
  for (int o = SG / 2; o > 0; o >>= 1) {
    NC += __shfl_xor(NC, o);
    NH += __shfl_xor(NH, o);
  }
  if (live && sub == 0) {
    if (cnt > scap) atomicOr(D.flags, F_OV_SHORT);
    D.sn[i] = min(cnt, scap);
    D.NCt[i] = (double)NC;
    D.NHt[i] = (double)NH;
  }
  // species-bucketed bond list: lane offsets by wave prefix sums, one LDS
  // add per wavefront and class, one global reservation per block and class
  // (same-address global atomics serialise: one per wavefront of 4 atoms
  // cost more than the whole kernel)
  __shared__ int s_cnt[3], s_base[3], s_max;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  const int nslot = live ? min(cnt, scap) : 0;   // slots sub, sub + SG of this atom are this lane's
  int nb[3] = {0, 0, 0};
  for (int t = sub; t < nslot; t += SG) {
    int q = s_cls[la][t];
    if (q >= 0) nb[q]++;
  }
  int base[3];
  for (int q = 0; q < 3; ++q) {
    int incl = nb[q];
    for (int o = 1; o < WAVE; o <<= 1) {
      int u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    int tot = __shfl(incl, WAVE - 1);
    int wofs = 0;
    if (lane == WAVE - 1 && tot) wofs = atomicAdd(&s_cnt[q], tot);
    base[q] = __shfl(wofs, WAVE - 1) + incl - nb[q];
  }
  int mx = wave_max(cnt);   // largest short-list count, one global update per block
  if (lane == 0 && mx > 0) atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x < 3 && s_cnt[threadIdx.x] > 0) s_base[threadIdx.x] = atomicAdd(&D.bcount[threadIdx.x], s_cnt[threadIdx.x]);
  if (threadIdx.x == 0 && s_max > 0) atomicMax(&D.stats[S_MAXSHORT], (unsigned long long)s_max);
  __syncthreads();
  for (int q = 0; q < 3; ++q) base[q] += s_base[q];
  for (int t = sub; t < nslot; t += SG) {
    int q = s_cls[la][t];
    if (q < 0) continue;
    int b = base[q]++;
    if (b < D.bcap) D.bonds[q * D.bcap + b] = make_int2(i, t);
    else atomicOr(D.flags, F_OV_BOND);
  }
}

// Atoms and bond slots along a path code starting at atom i.
struct PathInfo { int len; int at[4]; int slot[3]; };
__device__ __forceinline__ PathInfo decode_path(const Dev& D, int i, int code) {
  PathInfo pi;
  pi.len = code & 3;
  pi.at[0] = i;
  int a = i;
  for (int b = 0; b < pi.len; ++b) {
    int s = (code >> (2 + 5 * b)) & 31;
    pi.slot[b] = s;
    a = D.sj[a * D.scap + s];
    pi.at[b + 1] = a;
  }
  return pi;
}

// Path code of a path i -> k (slot q1 of i), -> m (slot q2 of k), -> t (slot
// q3 of m): the length in the low two bits, then 5 bits per slot.
__device__ __forceinline__ int path_code(int len, int q1, int q2 = 0, int q3 = 0) {
  return len | (q1 << 2) | (q2 << 7) | (q3 << 12);
}

// Largest weight product over the paths of at most three short bonds from i
// to j that repeat no atom, and the code of the first path attaining it in
// the order direct, one intermediate, two intermediates (slot order within
// each).  This is the sequential C_ij search of the paper (Sec. 4.3) for
// atoms whose path map does not fit in LDS; it visits the same paths as the
// map with the same multiplication order.
__device__ void path_search(const Dev& D, int i, int j, double& best, int& bcode) {
  const int S = D.scap;
  best = 0.0;
  bcode = 0;
  int ni = D.sn[i];
  for (int q1 = 0; q1 < ni; ++q1) {
    double w1 = D.sw[i * S + q1].x;
    if (D.sj[i * S + q1] == j && w1 > best) { best = w1; bcode = path_code(1, q1); }
  }
  for (int q1 = 0; q1 < ni; ++q1) {
    int k = D.sj[i * S + q1];
    double w1 = D.sw[i * S + q1].x;
    int nk = D.sn[k];
    for (int q2 = 0; q2 < nk; ++q2) {
      int m = D.sj[k * S + q2];
      if (m == i) continue;
      double w2 = w1 * D.sw[k * S + q2].x;
      if (m == j && w2 > best) { best = w2; bcode = path_code(2, q1, q2); }
    }
  }
  for (int q1 = 0; q1 < ni; ++q1) {
    int k = D.sj[i * S + q1];
    double w1 = D.sw[i * S + q1].x;
    int nk = D.sn[k];
    for (int q2 = 0; q2 < nk; ++q2) {
      int m = D.sj[k * S + q2];
      if (m == i) continue;
      double w2 = w1 * D.sw[k * S + q2].x;
      if (w2 <= 0.0) continue;
      int nm = D.sn[m];
      for (int q3 = 0; q3 < nm; ++q3) {
        int t = D.sj[m * S + q3];
        if (t != j || t == k) continue;
        double w3 = w2 * D.sw[m * S + q3].x;
        if (w3 > best) { best = w3; bcode = path_code(3, q1, q2, q3); }
      }
    }
  }
}

// Gradient of E with respect to the path bonds, given dE/dprod.  `half`
// halves the contribution to every atom except the path start (full-list LJ
// visits each pair from both ends).
template <typename R, typename AC>
__device__ void path_grad(const Dev& D, const PathInfo& pi, R GP, double scale_all, double scale_start, AC& acc) {
  using A = typename AC::A;
  R w[3], dw[3], rl[3];
  V3<R> rv[3];
  for (int b = 0; b < pi.len; ++b) {
    int a = pi.at[b], s = pi.slot[b];
    rv[b] = nbr_vec<R>(D, a, s, rl[b]);
    double2 wd = D.sw[a * D.scap + s];
    w[b] = (R)wd.x;
    dw[b] = (R)wd.y;
  }
  const A sall = (A)scale_all;
  for (int b = 0; b < pi.len; ++b) {
    if (dw[b] == (R)0) continue;
    R others = 1;
    for (int c = 0; c < pi.len; ++c) if (c != b) others *= w[c];
    V3<R> g = (GP * others * dw[b] / rl[b]) * rv[b];
    A gx = g.x, gy = g.y, gz = g.z;
    int a = pi.at[b], c = pi.at[b + 1];
    A sa = (b == 0) ? (A)scale_start : sall;
    acc.force(a, sa * gx, sa * gy, sa * gz);
    if (b + 1 < pi.len || scale_all == 1.0) acc.force(c, -sall * gx, -sall * gy, -sall * gz);
    A rx = rv[b].x, ry = rv[b].y, rz = rv[b].z;
    acc.W[0] -= sall * rx * gx; acc.W[1] -= sall * ry * gy; acc.W[2] -= sall * rz * gz;
    acc.W[3] -= sall * rx * gy; acc.W[4] -= sall * rx * gz; acc.W[5] -= sall * ry * gz;
  }
}

// REBO pair + bond order + torsion, one lane per bond (Alg. 1 and 2 merged).
template <typename R, typename A>
__global__ __launch_bounds__(64) void k_bond(Dev D, const DevParams* __restrict__ Pp, int mask) {
  if (D.skip && *D.skip) return;
  __shared__ DevParams sP;
  stage_params(sP, Pp);
  const DevParams& P = sP;
  int n0 = D.bcount[0], n1 = D.bcount[1], n2 = D.bcount[2];
  n0 = min(n0, D.bcap); n1 = min(n1, D.bcap); n2 = min(n2, D.bcap);
  int total = n0 + n1 + n2;
  A er = 0, et = 0;
  AccT<A> acc;
  acc.init(fbuf<A>(D), -1, -1);
  extern __shared__ __align__(16) unsigned char stage_mem[];
  Stage<R> SG;
  SG.init(stage_mem);
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < total; g += gridDim.x * blockDim.x) {
    int seg = g < n0 ? 0 : (g < n0 + n1 ? 1 : 2);
    int off = g - (seg == 0 ? 0 : (seg == 1 ? n0 : n0 + n1));
    int2 bq = D.bonds[seg * D.bcap + off];
    int i = bq.x, slot = bq.y;
    int j = D.sj[i * D.scap + slot];
    R r;
    V3<R> rij = nbr_vec<R>(D, i, slot, r);
    double2 wd = D.sw[i * D.scap + slot];
    R wij = (R)wd.x, dwij = (R)wd.y;
    int p = seg;
    SG.fill(D, i, j);
    acc.i = i; acc.j = j;
    for (int c = 0; c < 3; ++c) acc.fi[c] = acc.fj[c] = 0;
    A er0 = er, et0 = et, W0[6];
    for (int c = 0; c < 6; ++c) W0[c] = acc.W[c];
    V3<R> gij = {0, 0, 0};
    R Gr = 0;
    const bool tors = (mask & AIREBO_TERM_TORSION) && p == 0;
    R GSdh = 0;   // dE/d(pi^dh dihedral sum), taken in the torsion's pass over the same loop
    if (mask & AIREBO_TERM_REBO) {
      const R ir = rcp_nr(r);
      R ea = (R)P.alpha[p];
      R eR = xexp(-ea * r) * (R)P.A[p];
      R VR = ((R)1 + (R)P.Q[p] * ir) * eR;
      R dVR = -((R)P.Q[p] * ir * ir) * eR - ea * VR;
      R VA = 0, dVA = 0;
      for (int m = 0; m < 3; ++m) {
        if (P.B[p][m] == 0.0) continue;
        R t = (R)P.B[p][m] * xexp(-(R)P.beta[p][m] * r);
        VA += t;
        dVA -= (R)P.beta[p][m] * t;
      }
      R Gb = -wij * VA;
      BondFwd<R> bf;
      R b = bond_order_fwd(P, D, SG, i, j, rij, r, false, bf, acc.st);
      bond_order_rev(P, D, SG, i, j, rij, r, false, bf, Gb, gij, acc, tors);
      if (tors && bf.dh) GSdh = Gb * bf.Tv;
      er += (A)(wij * (VR - b * VA));
      Gr += dwij * (VR - b * VA) + wij * (dVR - b * dVA);
    }
    if (tors) {
      R Sdh = 0, Et = 0, Gwij = 0;
      dihedral(P, D, SG, i, j, rij, r, wij, true, true, GSdh, Sdh, Et, gij, Gwij, acc);
      et += (A)Et;
      Gr += Gwij * dwij;
    }
    gij = gij + (Gr * rcp_nr(r)) * rij;
    acc.vec(i, j, rij, gij);
    acc.flush();
    if (D.nsys > 1) {
      double dv[9] = {(double)(er - er0), (double)(et - et0), 0.0};
      for (int c = 0; c < 6; ++c) dv[3 + c] = (double)(acc.W[c] - W0[c]);
      int sid = sys_of(D, i);
      for (int q = 0; q < 9; ++q)
        if (dv[q] != 0) atomic_add(&D.sys_acc[(size_t)sid * A_N + A_EREBO + q], dv[q]);
    }
  }
  double v15[15] = {(double)er, (double)et, 0.0, (double)acc.W[0], (double)acc.W[1], (double)acc.W[2],
                    (double)acc.W[3], (double)acc.W[4], (double)acc.W[5], 0.0, 0.0, 0.0, 0.0,
                    (double)acc.st[0], (double)acc.st[1]};
  block_reduce_add<15>(v15, D.acc + A_EREBO);  // A_EREBO .. A_SPL64
}

template <typename R>
__device__ __forceinline__ void lj_pair(const DevParams& P, int p, R r, R& V, R& dV) {
  const R ir = rcp_nr(r);
  R s = (R)P.sigma[p] * ir;
  R s2 = s * s, s6 = s2 * s2 * s2;
  R e4 = (R)(4.0 * P.eps[p]);
  R v = e4 * (s6 * s6 - s6);
  R dv = e4 * ((R)-12 * s6 * s6 + (R)6 * s6) * ir;
  R isw = (R)P.inv_lj_sw;
  R t = (r - (R)(P.rc[p] - P.lj_sw)) * isw, dS;
  R S = Sw(t, dS);
  V = v * S;
  dV = dv * S + v * dS * isw;
}

// Append the n (<= 2 WAVE) deferred pairs staged in LDS by one wavefront to
// the queue segment of its block: one reservation, coalesced stores.
// Returns 0 (the staging buffer is empty again).
__device__ __forceinline__ int flush_deferred(const Dev& D, int4* buf, int n) {
  int lane = threadIdx.x & (WAVE - 1);
  int seg = blockIdx.x & (NSEG - 1);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int base = 0;
  if (lane == 0) base = atomicAdd(D.qcount + seg * QSTRIDE, n);
  base = __shfl(base, 0);
  for (int k = lane; k < n; k += WAVE) {
    int slot = base + k;
    if (slot < D.qcap) D.q[(size_t)seg * D.qcap + slot] = buf[k];
    else atomicOr(D.flags, F_OV_QUEUE);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return 0;
}

// The same LJ pair term from r^2, for plain pairs: energy V and
// G = (dV/dr) / r.  One division (1 / r^2); the square root is taken only
// inside the outer switching shell (rc - lj_sw < r < rc).
template <typename R>
__device__ __forceinline__ void lj_pair_r2(const DevParams& P, int p, R r2, R& V, R& G) {
  R ir2 = (R)1 / r2;
  R sg = (R)P.sigma[p];
  R s2 = sg * sg * ir2;
  R s6 = s2 * s2 * s2;
  R e4 = (R)(4.0 * P.eps[p]);
  R v = e4 * (s6 * s6 - s6);
  R gv = e4 * ((R)-12 * s6 * s6 + (R)6 * s6) * ir2;
  R r0 = (R)(P.rc[p] - P.lj_sw);
  if (r2 > r0 * r0) {
    R r = sqrt(r2);
    R isw = (R)P.inv_lj_sw, dS;
    R S = Sw((r - r0) * isw, dS);
    V = v * S;
    G = gv * S + v * dS * isw / r;
  } else {
    V = v;
    G = gv;
  }
}

// Morse pair term of the AIREBO-M variant, eps [e^{-2a(r-re)} - 2 e^{-a(r-re)}],
// under the same outer cutoff switch as the LJ term: V and dV/dr.
template <typename R>
__device__ __forceinline__ void morse_pair(const DevParams& P, int p, R r, R& V, R& dV) {
  R a = (R)P.m_alpha[p];
  R ex = xexp(-a * (r - (R)P.m_re[p]));
  R e = (R)P.m_eps[p];
  R v = e * (ex * ex - (R)2 * ex);
  R dv = (R)2 * a * e * (ex - ex * ex);
  R isw = (R)P.inv_lj_sw;
  R t = (r - (R)(P.rc[p] - P.lj_sw)) * isw, dS;
  R S = Sw(t, dS);
  V = v * S;
  dV = dv * S + v * dS * isw;
}

// Per-species-pair constants of the plain pair term, read once per kernel
// (uniform loads) and selected per lane by the pair class p, so that the
// pair loop issues no parameter load that depends on a gathered position.
struct PairConst {
  double rc2[3], sg2[3], e4[3], r0[3], rlj2[3];
  double rconn2, isw;
  __device__ void load(const DevParams& P) {
    for (int p = 0; p < 3; ++p) {
      rc2[p] = P.rc2[p];
      sg2[p] = P.sigma[p] * P.sigma[p];
      e4[p] = 4.0 * P.eps[p];
      r0[p] = P.rc[p] - P.lj_sw;
      rlj2[p] = P.rljmax[p] * P.rljmax[p];
    }
    rconn2 = P.r_conn * P.r_conn;
    isw = 1.0 / P.lj_sw;
  }
};
__device__ __forceinline__ double sel3(const double (&a)[3], int p) { return p == 0 ? a[0] : (p == 1 ? a[1] : a[2]); }


// Plain LJ pair from r^2 with the pair-class constants already selected:
// sg2 = sigma^2, e4 = 4 eps, r0 = start of the outer switch.
template <typename R>
__device__ __forceinline__ void lj_pair_r2c(R r2, R sg2, R e4, R r0, R isw, R& V, R& G) {
  R ir2 = rcp_nr(r2);
  R s2 = sg2 * ir2;
  R s6 = s2 * s2 * s2;
  R v = e4 * (s6 * s6 - s6);
  R gv = e4 * ((R)-12 * s6 * s6 + (R)6 * s6) * ir2;
  if (r2 > r0 * r0) {
    R ir = rsq_nr(r2);
    R r = r2 * ir;
    R dS;
    R S = Sw((r - r0) * isw, dS);
    V = v * S;
    G = gv * S + v * dS * isw * ir;
  } else {
    V = v;
    G = gv;
  }
}

// The van der Waals pair term: Lennard-Jones, or Morse with M (AIREBO-M).
template <typename R, bool M>
__device__ __forceinline__ void vdw_pair(const DevParams& P, int p, R r, R& V, R& dV) {
  if constexpr (M) morse_pair<R>(P, p, r, V, dV);
  else lj_pair<R>(P, p, r, V, dV);
}
// From r^2 for plain pairs: V and G = (dV/dr) / r.
template <typename R, bool M>
__device__ __forceinline__ void vdw_pair_r2(const DevParams& P, int p, R r2, R& V, R& G) {
  if constexpr (M) {
    R r = xsqrt(r2), dV;
    morse_pair<R>(P, p, r, V, dV);
    G = dV / r;
  } else {
    lj_pair_r2<R>(P, p, r2, V, G);
  }
}

// LJ term (Alg. 3), near pairs: one wavefront per atom over the near part of
// its list (the far part is k_ljf's).
//
// The wavefront first maps every atom reachable from i over at most three
// short bonds (no atom repeated) into LDS, with the weight product of the
// path and the path itself (the reversed C_ij search: map once per atom, then
// look up per pair).  Candidates are kept per path; a lookup takes the
// largest product over the candidates of an atom (first one on ties, direct
// before one intermediate before two).  Then, over the near list, pairs
// beyond 3 max R2 are plain LJ; nearer pairs look up C_ij: C = 0 is skipped,
// C = 1 outside the S_r range is plain LJ, and every other pair (0 < C < 1 or
// inside the S_r range) is deferred to a queue that k_bstar evaluates in
// full.  Each pair is seen from both ends: each end adds half the energy and
// virial and the full force on its own atom.
// Minimum waves per SIMD asked of the compiler for the near LJ kernel (the
// wave-uniform atom data in scalar registers): FP64 and mixed precision fit
// seven (72 and 64 VGPRs) without spilling, where eight would spill; single
// precision eight (63 VGPRs); the Morse form (a square root and an
// exponential more per pair) five (96 VGPRs).
template <typename R, typename A, bool M>
struct LjWaves {
  static constexpr int value = M ? 5 : (std::is_same<A, float>::value ? 8 : 7);
};

template <typename R, typename A, bool M>
__global__ __launch_bounds__(LJ_BLOCK) __attribute__((amdgpu_waves_per_eu(LjWaves<R, A, M>::value, 8))) void k_lj(
    Dev D, const DevParams* __restrict__ Pp) {
  if (D.skip && *D.skip) return;
  const DevParams& P = *Pp;
  __shared__ int c_atom[LJ_BLOCK / WAVE][PCAP];
  __shared__ int c_code[LJ_BLOCK / WAVE][PCAP];
  __shared__ int c_k[LJ_BLOCK / WAVE][PCAP];
  __shared__ double c_prod[LJ_BLOCK / WAVE][PCAP];
  // candidate lookup by atom: open addressing; the value packs the product's
  // bits (low 6 cleared) above 63 - candidate index, so an atomic max keeps
  // the largest product and, on ties, the first candidate
  __shared__ int h_key[LJ_BLOCK / WAVE][HCAP];
  __shared__ unsigned long long h_val[LJ_BLOCK / WAVE][HCAP];
  // deferred pairs of the wavefront, appended to the queue in one reservation
  // when WAVE more might not fit and at the end
  __shared__ int4 dq[LJ_BLOCK / WAVE][2 * WAVE];
  // per-pair-class constants of the plain pair term, read by lane-dependent
  // class index from LDS
  __shared__ PairConst K;
  if (threadIdx.x == 0) K.load(P);
  __syncthreads();
  int ndq = 0;
  int lane = threadIdx.x & (WAVE - 1);
  int wv = threadIdx.x / WAVE;
  // one atom per wavefront: the index is wave-uniform, and saying so keeps
  // the atom's position, box, list base and count in scalar registers
  int i = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
  unsigned long long below = lanes_below();
  A e = 0;
  A fi[3] = {0, 0, 0}, W[6] = {0, 0, 0, 0, 0, 0};
  unsigned n_in = 0, n_c0 = 0;   // per-lane counts (at most the list length)
  int n_srch = 0;   // pairs of this wavefront sent to the sequential C_ij search
  if (i < D.n) {
    double4 xi = D.x[i];
    int si = __double2int_rn(xi.w);
    const SysBox& B = box_of(D, i);
    const double Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
    // ---- path map.  Level 1: one lane per short neighbour k of i.
    int ncand = 0;
    bool ovf;   // more candidates than the map holds: near pairs go to the sequential search
    {
      const int S = D.scap, sl = D.slog2;
      const int ni = D.sn[i];
      {
        int k = -1;
        double w1 = 0;
        if (lane < ni) {
          k = D.sj[i * S + lane];
          w1 = D.sw[i * S + lane].x;
        }
        bool c1 = k >= 0 && w1 > 0.0;
        unsigned long long b1 = __ballot(c1);
        if (c1) {
          int pos = __popcll(b1 & below);
          c_atom[wv][pos] = k; c_prod[wv][pos] = w1; c_code[wv][pos] = path_code(1, lane); c_k[wv][pos] = i;
        }
        ncand = __popcll(b1);
      }
      const int n2start = ncand;
      // level 2: one lane per (q1, q2)
      for (int base = 0; base < (ni << sl); base += WAVE) {
        int t = base + lane, q1 = t >> sl, q2 = t & (S - 1);
        int k = -1, m = -1;
        double w2 = 0;
        if (q1 < ni) {
          k = D.sj[i * S + q1];
          double w1 = D.sw[i * S + q1].x;
          if (q2 < D.sn[k]) {
            m = D.sj[k * S + q2];
            w2 = w1 * D.sw[k * S + q2].x;
          }
        }
        bool c2 = m >= 0 && m != i && w2 > 0.0;
        unsigned long long b2 = __ballot(c2);
        if (c2) {
          int pos = ncand + __popcll(b2 & below);
          if (pos < PCAP) {
            c_atom[wv][pos] = m; c_prod[wv][pos] = w2; c_code[wv][pos] = path_code(2, q1, q2); c_k[wv][pos] = k;
          }
        }
        ncand += __popcll(b2);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int n2end = min(ncand, PCAP);
      // ---- level 3: one lane per (level-2 candidate, q3)
      for (int base = n2start << sl; base < (n2end << sl); base += WAVE) {
        int c = (base + lane) >> sl, q3 = (base + lane) & (S - 1);
        bool c3 = false;
        int t = -1, code = 0;
        double w3 = 0;
        if (c < n2end) {
          int mm = c_atom[wv][c], kk = c_k[wv][c];
          if (q3 < D.sn[mm]) {
            t = D.sj[mm * S + q3];
            w3 = c_prod[wv][c] * D.sw[mm * S + q3].x;
            code = (c_code[wv][c] & ~3) | 3 | (q3 << 12);
            c3 = t != i && t != kk && w3 > 0.0;
          }
        }
        unsigned long long b3 = __ballot(c3);
        if (c3) {
          int pos = ncand + __popcll(b3 & below);
          if (pos < PCAP) { c_atom[wv][pos] = t; c_prod[wv][pos] = w3; c_code[wv][pos] = code; }
        }
        ncand += __popcll(b3);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      ovf = ncand > PCAP;
      ncand = min(ncand, PCAP);
      for (int k = lane; k < HCAP; k += WAVE) { h_key[wv][k] = -1; h_val[wv][k] = 0ull; }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < ncand && !ovf) {   // PCAP == WAVE: one candidate per lane
        int a = c_atom[wv][lane];
        unsigned long long v = ((unsigned long long)__double_as_longlong(c_prod[wv][lane]) & ~63ull) |
                               (unsigned long long)(63 - lane);
        int h = hslot(a);
        for (int probe = 0; probe < HCAP; ++probe) {
          int old = atomicCAS(&h_key[wv][h], -1, a);
          if (old == -1 || old == a) { atomicMax(&h_val[wv][h], v); break; }
          h = (h + 1) & (HCAP - 1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    // ---- pair loop; the list entries of the next block of 64 are loaded
    // while this block is evaluated
    int nl = min(D.lj_n[i], D.lj_cap);
    const unsigned* list = D.lj_e + (size_t)i * D.lj_cap;
    unsigned ent_n = lane < nl ? list[lane] : 0u;
    for (int base = 0; base < nl; base += WAVE) {
      int e0 = base + lane;
      bool push = false;
      int j = 0, code = 0, pcode = 0;
      unsigned ent = ent_n;
      if (e0 + WAVE < nl) ent_n = list[e0 + WAVE];
      if (e0 < nl) {
        j = (int)(ent & 0x7FFFFFFu);
        code = (int)(ent >> 27);
        double4 xj = D.x[j];
        // relative vector in A: single precision forms it from FP32 positions
        A dx = (A)xj.x - (A)xi.x + (A)((code / 9 - 1) * Lx);
        A dy = (A)xj.y - (A)xi.y + (A)(((code / 3) % 3 - 1) * Ly);
        A dz = (A)xj.z - (A)xi.z + (A)((code % 3 - 1) * Lz);
        A r2 = dx * dx + dy * dy + dz * dz;
        int p = si + __double2int_rn(xj.w);
        if ((double)r2 < sel3(K.rc2, p)) {
          if (i < j) ++n_in;
          bool plain = true;
          if (r2 < K.rconn2 && ovf) {
            // path map incomplete: the deferred kernel searches C_ij for this
            // pair and takes this end's share of it
            push = true;
            pcode = -1;
            plain = false;
            ++n_srch;
          } else if (r2 < K.rconn2) {
            double prod = 0.0;
            int h = hslot(j);
            for (int probe = 0; probe < HCAP; ++probe) {
              int key = h_key[wv][h];
              if (key == j) {
                int c = 63 - (int)(h_val[wv][h] & 63ull);
                prod = c_prod[wv][c];
                pcode = c_code[wv][c];
                break;
              }
              if (key < 0) break;
              h = (h + 1) & (HCAP - 1);
            }
            if (prod >= 1.0) {
              if (i < j) ++n_c0;
              plain = false;
            } else if (prod > 0.0 || r2 < sel3(K.rlj2, p)) {
              push = i < j;
              plain = false;
            }
          }
          if (plain) {
            // pair arithmetic in R on the relative vector; accumulation in A
            // (energy and virial halved once, at the end)
            R V, g;   // dE/dr_ij vector = g * d
            if constexpr (M) vdw_pair_r2<R, M>(P, p, (R)r2, V, g);
            else lj_pair_r2c<R>((R)r2, (R)sel3(K.sg2, p), (R)sel3(K.e4, p), (R)sel3(K.r0, p), (R)K.isw, V, g);
            e += (A)V;
            R fx = g * (R)dx, fy = g * (R)dy, fz = g * (R)dz;
            fi[0] += (A)fx; fi[1] += (A)fy; fi[2] += (A)fz;
            W[0] += (A)(fx * (R)dx); W[1] += (A)(fy * (R)dy); W[2] += (A)(fz * (R)dz);
            W[3] += (A)(fy * (R)dx); W[4] += (A)(fz * (R)dx); W[5] += (A)(fz * (R)dy);
          }
        }
      }
      // deferred pairs: staged in LDS, flushed when the next block might
      // not fit
      unsigned long long pm = __ballot(push);
      if (push) dq[wv][ndq + __popcll(pm & below)] = make_int4(i, j, code, pcode);
      ndq += __popcll(pm);
      if (ndq > WAVE) ndq = flush_deferred(D, dq[wv], ndq);
    }
  }
  if (ndq > 0) flush_deferred(D, dq[wv], ndq);
  for (int o = WAVE / 2; o > 0; o >>= 1) n_srch += __shfl_xor(n_srch, o);
  if (lane == 0 && n_srch > 0) atomicAdd(&D.stats[S_SLOW], (unsigned long long)n_srch);
  // reduce the force on atom i across the wavefront
  for (int c = 0; c < 3; ++c) {
    A s = fi[c];
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && i < D.n && s != 0) atomic_add(&fbuf<A>(D)[3 * i + c], s);
  }
  // each pair is seen from both ends: half the energy, minus half the virial
  double v9[9] = {0.5 * (double)e, -0.5 * (double)W[0], -0.5 * (double)W[1], -0.5 * (double)W[2],
                  -0.5 * (double)W[3], -0.5 * (double)W[4], -0.5 * (double)W[5], (double)n_in, (double)n_c0};
  if (D.nsys > 1) sys_add<7>(D, i < D.n ? sys_of(D, i) : 0, *(const double(*)[7])v9, A_ELJ, i < D.n);
  block_reduce_add<9>(v9, D.acc + A_ELJ);   // A_ELJ, A_VIR..A_VIR+5, A_NIN, A_NC0 are consecutive
}

// Far LJ pairs: beyond 3 max R2 + skin at the list build, so beyond 3 max R2
// for the list's lifetime, where no path of three short bonds reaches
// (C_ij = 1) and the S_r switch is 0: the plain pair term with its outer
// cutoff switch (Alg. 3 with C = 1, S_r = 0).  LJF_G lanes per atom take its
// entries in turn, LJF_U at a time, every list entry and position of the
// LJF_U requested before any is used, so that a wavefront keeps many
// position gathers in flight; no LDS path map, few registers, high
// occupancy.  Each pair is seen from both ends, as in the near kernel.
#ifndef LJF_UNROLL
#define LJF_UNROLL 2
#endif
#ifndef LJF_MIN_WAVES
#define LJF_MIN_WAVES 5
#endif
constexpr int LJF_G = 16, LJF_U = LJF_UNROLL, LJF_WAVES = LJF_MIN_WAVES;
// MI: every periodic side is at least twice the list cutoff plus twice the
// skin, so each listed pair stays closer than half a side and its relative
// vector is the minimum image (no shift code decoded).
template <typename R, typename A, bool M, bool MI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M ? 4 : LJF_WAVES, 8))) void k_ljf(
    Dev D, const DevParams* __restrict__ Pp) {
  if (D.skip && *D.skip) return;
  const DevParams& P = *Pp;
  __shared__ PairConst K;
  if (threadIdx.x == 0) K.load(P);
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int sub = lane & (LJF_G - 1);
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LJF_G);
  constexpr unsigned NONE = 0xFFFFFFFFu;   // no entry (a real entry has shift code <= 26)
  A e = 0;
  A fi[3] = {0, 0, 0}, W[6] = {0, 0, 0, 0, 0, 0};
  unsigned long long n_in = 0;
  if (i < D.n) {
    const double4 xi = D.x[i];
    const int si = __double2int_rn(xi.w);
    const SysBox& B = box_of(D, i);
    const double Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
    // minimum image: inverse sides of the periodic directions, 0 otherwise
    const A iLx = B.per[0] ? (A)B.invL[0] : (A)0, iLy = B.per[1] ? (A)B.invL[1] : (A)0,
            iLz = B.per[2] ? (A)B.invL[2] : (A)0;
    const int nl = min(D.lf_n[i], D.lf_cap);
    const unsigned* list = D.lf_e + (size_t)i * D.lf_cap;
    for (int k0 = sub; k0 < nl; k0 += LJF_G * LJF_U) {
      unsigned ent[LJF_U];
      double4 xj[LJF_U];
#pragma unroll
      for (int u = 0; u < LJF_U; ++u) {
        int k = k0 + u * LJF_G;
        ent[u] = k < nl ? list[k] : NONE;
      }
      // unconditional loads (a missing entry reads atom i's own position)
#pragma unroll
      for (int u = 0; u < LJF_U; ++u) xj[u] = D.x[ent[u] != NONE ? (int)(ent[u] & 0x7FFFFFFu) : i];
#pragma unroll
      for (int u = 0; u < LJF_U; ++u) {
        if (ent[u] == NONE) continue;
        const int j = (int)(ent[u] & 0x7FFFFFFu), code = (int)(ent[u] >> 27);
        A dx, dy, dz;
        if constexpr (MI) {
          dx = (A)xj[u].x - (A)xi.x;
          dy = (A)xj[u].y - (A)xi.y;
          dz = (A)xj[u].z - (A)xi.z;
          dx -= (A)Lx * xrint(dx * iLx);
          dy -= (A)Ly * xrint(dy * iLy);
          dz -= (A)Lz * xrint(dz * iLz);
        } else {
          dx = (A)xj[u].x - (A)xi.x + (A)((code / 9 - 1) * Lx);
          dy = (A)xj[u].y - (A)xi.y + (A)(((code / 3) % 3 - 1) * Ly);
          dz = (A)xj[u].z - (A)xi.z + (A)((code % 3 - 1) * Lz);
        }
        A r2 = dx * dx + dy * dy + dz * dz;
        int p = si + __double2int_rn(xj[u].w);
        if ((double)r2 < sel3(K.rc2, p)) {
          if (i < j) ++n_in;
          R V, g;   // dE/dr_ij vector = g * d
          if constexpr (M) vdw_pair_r2<R, M>(P, p, (R)r2, V, g);
          else lj_pair_r2c<R>((R)r2, (R)sel3(K.sg2, p), (R)sel3(K.e4, p), (R)sel3(K.r0, p), (R)K.isw, V, g);
          e += (A)V;
          R fx = g * (R)dx, fy = g * (R)dy, fz = g * (R)dz;
          fi[0] += (A)fx; fi[1] += (A)fy; fi[2] += (A)fz;
          W[0] += (A)(fx * (R)dx); W[1] += (A)(fy * (R)dy); W[2] += (A)(fz * (R)dz);
          W[3] += (A)(fy * (R)dx); W[4] += (A)(fz * (R)dx); W[5] += (A)(fz * (R)dy);
        }
      }
    }
  }
  // force on atom i: reduce over its LJF_G lanes
  for (int c = 0; c < 3; ++c) {
    A v = fi[c];
    for (int o = LJF_G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (sub == 0 && i < D.n && v != 0) atomic_add(&fbuf<A>(D)[3 * i + c], v);
  }
  double v16[16] = {0.5 * (double)e, -0.5 * (double)W[0], -0.5 * (double)W[1], -0.5 * (double)W[2],
                    -0.5 * (double)W[3], -0.5 * (double)W[4], -0.5 * (double)W[5]};
  v16[A_NINF - A_ELJ] = (double)n_in;   // far pairs inside the cutoff, counted apart from the near ones
  if (D.nsys > 1) sys_add<7>(D, i < D.n ? sys_of(D, i) : 0, *(const double(*)[7])v16, A_ELJ, i < D.n);
  block_reduce_add<16>(v16, D.acc + A_ELJ);   // A_ELJ .. A_NINF
}

// Deferred LJ pairs (0 < C_ij < 1, or inside the S_r range where the modified
// bond order b* enters through S_b): energy and the full gradient, including
// the path atoms of C_ij and, where 0 < t_b < 1, the b* neighbourhood.
template <typename R, typename A, bool M>
__global__ __launch_bounds__(64) void k_bstar(Dev D, const DevParams* __restrict__ Pp) {
  if (D.skip && *D.skip) return;
  __shared__ DevParams sP;
  stage_params(sP, Pp);
  const DevParams& P = sP;
  __shared__ int seg_start[NSEG + 1];
  if (threadIdx.x == 0) {
    int run = 0;
    for (int g = 0; g < NSEG; ++g) { seg_start[g] = run; run += min(D.qcount[g * QSTRIDE], D.qcap); }
    seg_start[NSEG] = run;
  }
  __syncthreads();
  int nq = seg_start[NSEG];
  A e = 0;
  AccT<A> acc;
  acc.init(fbuf<A>(D), -1, -1);
  unsigned long long ndsb = 0;
  unsigned long long nskip = 0, nc0 = 0;   // searched pairs that are not deferred pairs; of them with C_ij = 0
  unsigned long long nbstar = 0;           // evaluated pairs inside the S_r range (b* needed)
  extern __shared__ __align__(16) unsigned char stage_mem[];
  Stage<R> SG;
  SG.init(stage_mem);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nq; t += gridDim.x * blockDim.x) {
    int g = 0;
    while (seg_start[g + 1] <= t) ++g;
    int4 qe = D.q[(size_t)g * D.qcap + (t - seg_start[g])];
    A W0[6];
    for (int c = 0; c < 6; ++c) W0[c] = acc.W[c];
    A e0 = e;
    int i = qe.x, j = qe.y, code = qe.z, pcode = qe.w;
    double4 xi = D.x[i], xj = D.x[j];
    const SysBox& B = box_of(D, i);
    // LJ part, C_ij and the switches in A (FP64, or FP32 in single precision)
    A dx = (A)xj.x - (A)xi.x + (A)((code / 9 - 1) * B.L[0]);
    A dy = (A)xj.y - (A)xi.y + (A)(((code / 3) % 3 - 1) * B.L[1]);
    A dz = (A)xj.z - (A)xi.z + (A)((code % 3 - 1) * B.L[2]);
    int p = __double2int_rn(xi.w) + __double2int_rn(xj.w);
    A r2 = dx * dx + dy * dy + dz * dz;
    A r = r2 * rsq_nr(r2);
    acc.i = i; acc.j = j;
    for (int c = 0; c < 3; ++c) acc.fi[c] = acc.fj[c] = 0;
    A V, dV;
    vdw_pair<A, M>(P, p, r, V, dV);
    bool evaluate = true;
    if (pcode < 0) {
      // sequential C_ij search for an atom whose path map overflowed; this
      // end classifies the pair as the map would have
      double best;
      path_search(D, i, j, best, pcode);
      if (best >= 1.0) {                                   // C_ij = 0
        if (i < j) ++nc0;
        evaluate = false;
      } else if (best > 0.0 || (double)r2 < P.rljmax[p] * P.rljmax[p]) {
        evaluate = i < j;                                   // a deferred pair: the lower index evaluates it
      } else {                                              // a plain pair: this end's half
        A G = dV * rcp_nr(r);
        e += (A)0.5 * V;
        A g3[3] = {G * dx, G * dy, G * dz};
        for (int c = 0; c < 3; ++c) acc.fi[c] += g3[c];
        acc.W[0] -= (A)0.5 * dx * g3[0]; acc.W[1] -= (A)0.5 * dy * g3[1]; acc.W[2] -= (A)0.5 * dz * g3[2];
        acc.W[3] -= (A)0.5 * dx * g3[1]; acc.W[4] -= (A)0.5 * dx * g3[2]; acc.W[5] -= (A)0.5 * dy * g3[2];
        acc.flush();
        evaluate = false;
      }
      if (!evaluate) ++nskip;
    }
    if (evaluate) {
      A prod = 0;
      PathInfo pi;
      pi.len = 0;
      if (pcode) {
        pi = decode_path(D, i, pcode);
        prod = 1;
        for (int b = 0; b < pi.len; ++b) prod *= (A)D.sw[pi.at[b] * D.scap + pi.slot[b]].x;
      }
      A C = (A)1 - prod;
      A dSr;
      A Sr = Sw((r - (A)P.sigma[p]) * (A)P.inv_rlj[p], dSr);
      dSr *= (A)P.inv_rlj[p];
      V3<R> rij = {(R)dx, (R)dy, (R)dz};
      V3<R> gij = {0, 0, 0};
      A Sb = 1, dSb = 0;
      BondFwd<R> bf;
      if (Sr > (A)0) {
        ++nbstar;
        SG.fill(D, i, j);
        R bs = bond_order_fwd(P, D, SG, i, j, rij, (R)r, true, bf, acc.st);
        A inv_b = (A)P.inv_db[p];
        Sb = Sw(((A)bs - (A)P.bmin[p]) * inv_b, dSb);
        dSb *= inv_b;
      }
      A Qf = Sr * Sb + (A)1 - Sr;
      e += Qf * C * V;
      A Gr = (dSr * Sb - dSr) * C * V + Qf * C * dV;
      if (dSb != (A)0) {   // the reverse pass reuses the forward state
        ++ndsb;
        R Gb = (R)(Sr * dSb * C * V);
        bond_order_rev(P, D, SG, i, j, rij, (R)r, true, bf, Gb, gij, acc);
      }
      if (prod > (A)0) path_grad<A>(D, pi, -Qf * V, 1.0, 1.0, acc);
      gij = gij + (R)(Gr * rcp_nr(r)) * rij;
      acc.vec(i, j, rij, gij);
      acc.flush();
    }
    if (D.nsys > 1) {
      double dv[7] = {(double)(e - e0)};
      for (int c = 0; c < 6; ++c) dv[1 + c] = (double)(acc.W[c] - W0[c]);
      int sid = sys_of(D, i);
      for (int q = 0; q < 7; ++q)
        if (dv[q] != 0) atomic_add(&D.sys_acc[(size_t)sid * A_N + A_ELJ + q], dv[q]);
    }
  }
  __syncthreads();
  double v15[15] = {(double)e, (double)acc.W[0], (double)acc.W[1], (double)acc.W[2], (double)acc.W[3],
                    (double)acc.W[4], (double)acc.W[5], 0.0, (double)nc0, (double)ndsb, 0.0,
                    (double)acc.st[0], (double)acc.st[1], (double)nskip, (double)nbstar};
  block_reduce_add<15>(v15, D.acc + A_ELJ);  // A_ELJ .. A_NBSTAR
}

// Maximum of per-atom counts into a statistics slot, and the sum of the
// counts clamped to `cap` into another (one atomic each per wavefront).
__global__ void k_max(const int* __restrict__ a, int n, int cap, unsigned long long* out_max,
                      unsigned long long* out_sum, unsigned long long* out_sum2) {
  int m = 0;
  unsigned long long sum = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    m = max(m, a[t]);
    sum += (unsigned long long)min(a[t], cap);
  }
  m = wave_max(m);
  sum = wave_sum(sum);
  if ((threadIdx.x & (WAVE - 1)) == 0 && m > 0) atomicMax(out_max, (unsigned long long)m);
  if ((threadIdx.x & (WAVE - 1)) == 0 && sum > 0) {
    atomicAdd(out_sum, sum);
    if (out_sum2) atomicAdd(out_sum2, sum);
  }
}

__global__ void k_finish(Dev D, double* energy, double* virial) {
  int t = threadIdx.x;
  __shared__ double tot[A_N];
  if (t < A_N) {
    double s = 0;
    for (int g = 0; g < NSLOT; ++g) s += D.acc[g * A_N + t];
    tot[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    if (D.nsys == 1) {
      energy[1] = tot[A_EREBO];
      energy[2] = tot[A_ELJ];
      energy[3] = tot[A_ETORS];
      energy[0] = tot[A_EREBO] + tot[A_ELJ] + tot[A_ETORS];
    }
    unsigned long long nq = 0;
    for (int g = 0; g < NSEG; ++g) nq += (unsigned long long)min(D.qcount[g * QSTRIDE], D.qcap);
    D.stats[S_BSTAR] = (unsigned long long)tot[A_NBSTAR];
    D.stats[S_QUEUED] = nq - (unsigned long long)tot[A_NSKIP];
    D.stats[S_BONDS] = (unsigned long long)(D.bcount[0] + D.bcount[1] + D.bcount[2]);
    D.stats[S_INCUT] = (unsigned long long)(tot[A_NIN] + tot[A_NINF]);
    D.stats[S_INCUTF] = (unsigned long long)tot[A_NINF];
    D.stats[S_CIJ0] = (unsigned long long)tot[A_NC0];
    D.stats[S_DSB] = (unsigned long long)tot[A_NDSB];
    D.stats[S_SPL] = (unsigned long long)tot[A_SPL];
    D.stats[S_SPL64] = (unsigned long long)tot[A_SPL64];
    if (!isfinite(tot[A_EREBO] + tot[A_ELJ] + tot[A_ETORS])) atomicOr(D.flags, F_NONFINITE);
  }
  if (D.nsys == 1) {
    if (t < 6) virial[t] = tot[A_VIR + t];
    return;
  }
  for (int sid = t; sid < D.nsys; sid += blockDim.x) {
    const double* a = D.sys_acc + (size_t)sid * A_N;
    energy[4 * sid + 1] = a[A_EREBO];
    energy[4 * sid + 2] = a[A_ELJ];
    energy[4 * sid + 3] = a[A_ETORS];
    energy[4 * sid + 0] = a[A_EREBO] + a[A_ELJ] + a[A_ETORS];
    for (int q = 0; q < 6; ++q) virial[6 * sid + q] = a[A_VIR + q];
  }
}

// ---------------------------------------------------------------------------
// Velocity Verlet
// ---------------------------------------------------------------------------
constexpr double FTM = 1.0 / 103.642691;   // eV / (A amu) -> A / fs^2
constexpr double KB = 8.617333262e-5;

__global__ void k_kick(Dev D, double* vel, double m0, double m1, double dt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double ke = 0;
  if (i < D.n) {
    double m = __double2int_rn(D.x[i].w) == 0 ? m0 : m1;
    double im = FTM / m;
    for (int c = 0; c < 3; ++c) {
      double v = vel[3 * i + c] + 0.5 * dt * D.F[3 * i + c] * im;
      vel[3 * i + c] = v;
      ke += 0.5 * m * v * v / FTM;
    }
    // a step that diverges stops the run at the end of its chunk
    if (!isfinite(ke)) atomicOr(D.flags, F_NONFINITE);
  }
  double v1[1] = {ke};
  if (D.nsys > 1) sys_add<1>(D, i < D.n ? sys_of(D, i) : 0, v1, A_KE, i < D.n);
  block_reduce_add<1>(v1, D.acc + A_KE);
}

// Control block of an MD run: where k_thermo writes its rows.  It lives in
// device memory and is written by the host before a run's replays, so the
// captured step does not depend on the run's output buffer.
struct MdCtl {
  double* thermo;   // [nrows][nsys][THERMO_W] or null
  int every;        // a row every `every` steps (0: none)
  int nrows;
};
constexpr int THERMO_W = 7;
constexpr double EV_A3_TO_BAR = 1.602176634e6;

// Thermo rows {step, PE, KE, Etot, T, rebuilds, P}: one row per system and
// output step ([row][nsys][THERMO_W]); one block.  P (bar) = (2 KE + tr W) /
// (3 V), defined for systems periodic in all three directions (0 otherwise).
__device__ void thermo_rows(const Dev& D, const MdCtl* __restrict__ ctl) {
  int s = *D.step;
  double* thermo = ctl->thermo;
  int every = ctl->every, nrows = ctl->nrows;
  __syncthreads();
  if (thermo && every > 0 && s % every == 0 && s / every < nrows) {
    for (int sid = threadIdx.x; sid < D.nsys; sid += blockDim.x) {
      double pe = 0, ke = 0, w = 0;
      int na = D.sys[sid].natoms;
      if (D.nsys == 1) {
        for (int g = 0; g < NSLOT; ++g) {
          const double* a = D.acc + g * A_N;
          pe += a[A_EREBO] + a[A_ELJ] + a[A_ETORS];
          ke += a[A_KE];
          w += a[A_VIR] + a[A_VIR + 1] + a[A_VIR + 2];
        }
      } else {
        const double* a = D.sys_acc + (size_t)sid * A_N;
        pe = a[A_EREBO] + a[A_ELJ] + a[A_ETORS];
        ke = a[A_KE];
        w = a[A_VIR] + a[A_VIR + 1] + a[A_VIR + 2];
      }
      const SysBox& B = D.sys[sid];
      bool per = B.per[0] && B.per[1] && B.per[2];
      double* row = thermo + THERMO_W * ((size_t)(s / every) * D.nsys + sid);
      row[0] = s;
      row[1] = pe;
      row[2] = ke;
      row[3] = pe + ke;
      row[4] = na > 1 ? 2.0 * ke / ((3.0 * na - 3.0) * KB) : 0.0;
      row[5] = (double)D.stats[S_REBUILD];
      row[6] = per ? (2.0 * ke + w) / (3.0 * B.L[0] * B.L[1] * B.L[2]) * EV_A3_TO_BAR : 0.0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *D.step = s + 1;
}

__global__ void k_thermo(Dev D, const MdCtl* __restrict__ ctl) {
  if (blockIdx.x == 0) thermo_rows(D, ctl);
}

// First half kick and drift of a step.  Block 0 first writes the thermo row
// of the state the previous step ended in (its sums are complete: a kernel
// boundary lies between) and then clears the sums for this step; the
// forces used here are zeroed by their atoms' threads, the bond and queue
// counters by any thread (the force chain of a step that starts here needs
// no separate zeroing).  A displacement beyond half the skin since the last
// build flags a rebuild.
__global__ void k_kick_drift(Dev D, double* vel, double m0, double m1, double dt, double half_skin2,
                             const MdCtl* __restrict__ ctl) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    thermo_rows(D, ctl);
    __syncthreads();
    for (int k = threadIdx.x; k < NSLOT * A_N; k += blockDim.x) D.acc[k] = 0;
    if (D.nsys > 1)
      for (int k = threadIdx.x; k < D.nsys * A_N; k += blockDim.x) D.sys_acc[k] = 0;
  }
  if (i < 3) D.bcount[i] = 0;
  if (i < NSEG) D.qcount[i * QSTRIDE] = 0;
  if (i >= D.n) return;
  double4 x = D.x[i];
  double im = FTM / (__double2int_rn(x.w) == 0 ? m0 : m1);
  double v[3];
  for (int c = 0; c < 3; ++c) v[c] = vel[3 * i + c] + 0.5 * dt * D.F[3 * i + c] * im;
  x.x += dt * v[0]; x.y += dt * v[1]; x.z += dt * v[2];
  for (int c = 0; c < 3; ++c) { vel[3 * i + c] = v[c]; D.F[3 * i + c] = 0; }
  D.x[i] = x;
  double4 xr = D.xref[i];
  double ddx = x.x - xr.x, ddy = x.y - xr.y, ddz = x.z - xr.z;
  if (ddx * ddx + ddy * ddy + ddz * ddz > half_skin2) atomicOr(D.flags, F_REBUILD);
}

__global__ void k_store(Dev D, double* pos) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.n) return;
  double4 x = D.x[i];
  pos[3 * i] = x.x; pos[3 * i + 1] = x.y; pos[3 * i + 2] = x.z;
}

__global__ void k_set_flags(Dev D, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *D.flags = v;
}

// ---------------------------------------------------------------------------
// Work area of the allocation-free evaluation (airebo_compute_static): every
// buffer of one evaluation of up to STATIC_MAX_ATOMS atoms, carved out of one
// file-scope device array at fixed offsets.
// ---------------------------------------------------------------------------
constexpr int64_t STATIC_MAX_ATOMS = 8192;
constexpr int64_t STATIC_LJ_ENTRIES = STATIC_MAX_ATOMS * 224;   // near LJ entries (224 per atom at the maximum)
constexpr int64_t STATIC_LF_ENTRIES = STATIC_MAX_ATOMS * 384;   // far LJ entries (384 per atom at the maximum)
constexpr int64_t STATIC_MAX_CELLS = 32768;
constexpr int64_t STATIC_QUEUE = 16 * STATIC_MAX_ATOMS + 1024 * NSEG;   // deferred-pair queue entries
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct StaticLayout {
  size_t x, xref, xsort, cell_of, cell_count, cell_start, cell_cursor, cell_atoms, lj_n, lj_e, lf_n, lf_e, in_n, in_e,
      sn, sj, sd, sw, NCt, NHt, bcount, bonds, qcount, q, F32, acc, stats, flags, step, sys, total;
};
constexpr StaticLayout static_layout() {
  StaticLayout L{};
  size_t o = 0;
  const size_t N = STATIC_MAX_ATOMS, C = STATIC_MAX_CELLS;
  const size_t bcap = N * SCAP / 2 + 64;
  size_t* fields[] = {&L.x, &L.xref, &L.xsort, &L.cell_of, &L.cell_count, &L.cell_start, &L.cell_cursor,
                      &L.cell_atoms, &L.lj_n, &L.lj_e, &L.lf_n, &L.lf_e, &L.in_n, &L.in_e, &L.sn, &L.sj, &L.sd, &L.sw, &L.NCt,
                      &L.NHt, &L.bcount, &L.bonds, &L.qcount, &L.q, &L.F32, &L.acc, &L.stats, &L.flags, &L.step,
                      &L.sys};
  const size_t bytes[] = {32 * N, 32 * N, 16 * N, 4 * N, 4 * C, 4 * (C + 1), 4 * C, 4 * N, 4 * N,
                          4 * (size_t)STATIC_LJ_ENTRIES, 4 * N, 4 * (size_t)STATIC_LF_ENTRIES, 4 * N, 4 * N * ICAP, 4 * N, 4 * N * SCAP, 32 * N * SCAP,
                          16 * N * SCAP, 8 * N, 8 * N, 16, 8 * 3 * bcap, 4 * NSEG * QSTRIDE,
                          16 * (size_t)STATIC_QUEUE, 12 * N, 8 * NSLOT * A_N, 8 * S_N, 16, 16, sizeof(SysBox)};
  for (size_t k = 0; k < sizeof(bytes) / sizeof(bytes[0]); ++k) {
    *fields[k] = o;
    o += al256(bytes[k]);
  }
  L.total = o;
  return L;
}
constexpr StaticLayout kStatic = static_layout();
static_assert(kStatic.total < (size_t)32 << 20, "static work area stays under 32 MiB");

// The work area itself.  Host code never uses this name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kStatic.total];

// Store one system box in device memory (passed by value: no host copy).
__global__ void k_put_box(SysBox* dst, SysBox b) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = b;
}

}  // namespace airebo

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
using namespace airebo;

namespace {
thread_local std::string g_err;
// device address of the static work area, per device ordinal (set at context creation)
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(AIREBO_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_) + " (" + \
                                       std::to_string((int)e_) + ")");                         \
  } while (0)

template <typename T>
int grow(T*& p, size_t& cap, size_t need) {
  if (need <= cap && p) return 0;
  if (p) hipFree(p);
  p = nullptr;
  size_t c = std::max<size_t>(need, 1);
  hipError_t e = hipMalloc((void**)&p, c * sizeof(T));
  if (e != hipSuccess) { cap = 0; return fail(AIREBO_E_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e)); }
  cap = c;
  return 0;
}
}  // namespace

struct airebo_ctx {
  airebo_options opt;
  DevParams P;
  DevParams* dP = nullptr;
  double* dtri = nullptr;
  Dev D;
  int64_t n = 0;
  int lj_cap = 0;
  // buffers and capacities
  double4 *x = nullptr, *xref = nullptr;
  float4* xsort = nullptr;
  size_t cx = 0, cxr = 0, cxs = 0;
  hipStream_t side = nullptr;     // second stream: bonded terms run beside the LJ chain
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_cursor = nullptr, *cell_atoms = nullptr;
  size_t c_of = 0, c_cc = 0, c_cs = 0, c_cu = 0, c_ca = 0;
  int* lj_n = nullptr;
  size_t c_ljn = 0;
  unsigned* lj_e = nullptr;
  size_t c_lje = 0;
  int lf_cap = 0;
  int* lf_n = nullptr;
  size_t c_lfn = 0;
  unsigned* lf_e = nullptr;
  size_t c_lfe = 0;
  int *in_n = nullptr, *in_e = nullptr, *sn = nullptr, *sj = nullptr;
  size_t c_inn = 0, c_ine = 0, c_sn = 0, c_sj = 0;
  double4* sd = nullptr;
  size_t c_sd = 0;
  double2* sw = nullptr;
  size_t c_sw = 0;
  double *NCt = nullptr, *NHt = nullptr;
  size_t c_nc = 0, c_nh = 0;
  int* bcount = nullptr;
  size_t c_bc = 0;
  int2* bonds = nullptr;
  size_t c_b = 0;
  int* qcount = nullptr;
  size_t c_qc = 0;
  int4* q = nullptr;
  size_t c_q = 0;
  double* F = nullptr;
  size_t c_F = 0;
  float* F32 = nullptr;   // single precision only
  size_t c_F32 = 0;
  double* acc = nullptr;
  size_t c_acc = 0;
  unsigned long long* stats = nullptr;
  size_t c_st = 0;
  int* flags = nullptr;
  size_t c_fl = 0;
  int* step = nullptr;
  size_t c_stp = 0;
  // device staging of airebo_compute_host
  double* hx = nullptr;      // positions [3n], then energy [4], virial [6], forces [3n]
  int* hs = nullptr;         // species [n]
  size_t c_hx = 0, c_hs = 0;
  unsigned long long host_stats[S_N] = {};
  // batch description
  int ncell = 0;
  std::vector<SysBox> hsys;
  std::vector<int> hatom_sys;
  SysBox* dsys = nullptr;
  size_t c_dsys = 0;
  int* atom_sys = nullptr;
  size_t c_asys = 0;
  double* sys_acc = nullptr;
  size_t c_sacc = 0;
  // deferred-pair queue entries reserved per atom, short-list and
  // intermediate-list entries per atom (all grow on overflow)
  int q_per_atom = 8;
  int scap = SCAP;
  int icap = ICAP;
  // capacity growths of the current call or MD session (statistics slot S_REGROW)
  unsigned long long regrow = 0;
  // molecular-dynamics session (airebo_md_*): the run's parameters, its
  // device state and save area, and the captured step
  struct Md {
    bool on = false;
    int nsys = 0;
    std::vector<int64_t> off;
    std::vector<double> boxes;
    std::vector<int32_t> pers;
    double m0 = 0, m1 = 0, dt = 0;
    std::function<void(hipStream_t, bool)> forces;   // one force evaluation (bool: zero the sums first)
    const int* skip = nullptr;                       // surrogate: flag that skips the AIREBO kernels
    double* vel = nullptr;                           // velocities [n][3]
    double4* xsave = nullptr;                        // state at the start of the current chunk
    double* vsave = nullptr;
    unsigned long long* ssave = nullptr;             // [S_N] statistics, then the step counter
    size_t c_vel = 0, c_xs = 0, c_vs = 0, c_ss = 0;
    void* ctl = nullptr;                             // device MdCtl
    double hctl[2] = {0, 0};                         // host image of the control block (pointer + two ints)
    double* scratch = nullptr;                       // energies / virials of the sizing evaluation
    size_t c_scr = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;
  } md;
  // per-kernel timing (profile mode)
  bool prof = false;
  struct Ev { int k; hipEvent_t a, b; };
  std::vector<Ev> ev;
};

// Launch a kernel; in profile mode bracket it with a pair of HIP events.
#define LAUNCH(C, KID, KER, GRID, BLOCK, STREAM, ...) LAUNCH_SHM(C, KID, KER, GRID, BLOCK, 0, STREAM, __VA_ARGS__)
#define LAUNCH_SHM(C, KID, KER, GRID, BLOCK, SHM, STREAM, ...)                            \
  do {                                                                                     \
    if ((C)->prof) {                                                                       \
      airebo_ctx::Ev e_{KID, nullptr, nullptr};                                            \
      (void)hipEventCreate(&e_.a);                                                         \
      (void)hipEventCreate(&e_.b);                                                         \
      (void)hipEventRecord(e_.a, STREAM);                                                  \
      hipLaunchKernelGGL(KER, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                      \
      (void)hipEventRecord(e_.b, STREAM);                                                  \
      (C)->ev.push_back(e_);                                                               \
    } else {                                                                               \
      hipLaunchKernelGGL(KER, GRID, BLOCK, SHM, STREAM, __VA_ARGS__);                      \
    }                                                                                      \
  } while (0)

extern "C" {

const char* airebo_last_error(void) { return g_err.c_str(); }

void airebo_options_default(airebo_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->precision = AIREBO_FP64;
  opt->term_mask = AIREBO_TERM_ALL;
  opt->skin = 1.0;
  opt->lj_cap = 0;
  opt->device = 0;
  opt->vdw = AIREBO_VDW_LJ;
}

}  // extern "C"

struct airebo_params_set {
  DevParams P;
  std::vector<double> tri;   // tricubic coefficients (host)
};

namespace {

int check_options(const airebo_options& o) {
  if (!(o.skin > 0.0 && o.skin < 5.0)) return fail(AIREBO_E_ARG, "skin must be in (0, 5) A");
  if (o.precision != AIREBO_FP64 && o.precision != AIREBO_MIXED && o.precision != AIREBO_SINGLE)
    return fail(AIREBO_E_ARG, "unknown precision");
  if (o.term_mask < 0 || o.term_mask > 7) return fail(AIREBO_E_ARG, "bad term mask");
  if (o.vdw != AIREBO_VDW_LJ && o.vdw != AIREBO_VDW_MORSE) return fail(AIREBO_E_ARG, "unknown van der Waals form");
  if (o.vdw == AIREBO_VDW_MORSE && o.precision != AIREBO_FP64)
    return fail(AIREBO_E_ARG, "the Morse (AIREBO-M) form is evaluated in FP64 only");
  if (o.lj_cap < 0 || o.lj_slack < 0 || o.queue_per_atom < 0 || o.queue_per_atom > 1024)
    return fail(AIREBO_E_ARG, "bad lj_cap, lj_slack or queue_per_atom");
  // the bond-order kernels are one wavefront per block (their LDS stage is
  // sized for 64 threads)
  auto okb = [](int b) { return b == 0 || b == 64; };
  auto oks = [](int b) { return b == 0 || b == 256 || b == 512 || b == 1024; };
  if (!okb(o.bond_block) || !okb(o.defer_block) || !oks(o.short_block) || o.bond_grid < 0)
    return fail(AIREBO_E_ARG, "launch shapes: bond and deferred blocks 0 or 64 threads; "
                              "short-list block 0 or 256, 512, 1024 threads");
  if (o.schedule < AIREBO_SCHED_AUTO || o.schedule > AIREBO_SCHED_FAR_AFTER_NEAR)
    return fail(AIREBO_E_ARG, "unknown force-kernel schedule");
  return 0;
}

// A context from validated parameters: upload, streams, events.
int ctx_create_impl(const DevParams& P, const std::vector<double>& tri, const airebo_options& o, airebo_ctx_t* out) {
  airebo_ctx* c = new airebo_ctx();
  c->opt = o;
  if (o.queue_per_atom > 0) c->q_per_atom = o.queue_per_atom;
  c->P = P;
  c->P.knot_delta = o.precision == AIREBO_SINGLE ? -1.0 : KNOT_DELTA;   // single: FP32 everywhere
  if (o.vdw == AIREBO_VDW_MORSE && !P.morse_ok) {
    delete c;
    return fail(AIREBO_E_PARAMS, "the parameter set has no Morse records (morse_eps_/morse_re_/morse_alpha_ CC, CH, HH)");
  }
  if (o.device < 0 || o.device >= kMaxDevices) {
    delete c;
    return fail(AIREBO_E_ARG, "device ordinal out of range");
  }
  hipError_t e = hipSetDevice(o.device);
  if (e == hipSuccess) {   // once per device, with that device current
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[o.device]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e == hipSuccess && !ptr) e = hipErrorInvalidSymbol;
      if (e == hipSuccess) g_static_ptr[o.device] = ptr;
    }
  }
  if (e == hipSuccess) e = hipMalloc((void**)&c->dtri, tri.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(c->dtri, tri.data(), tri.size() * sizeof(double), hipMemcpyHostToDevice);
  c->P.tri = c->dtri;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&c->dP, sizeof(DevParams));
  if (e == hipSuccess) e = hipMemcpy(c->dP, &c->P, sizeof(DevParams), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    std::string m = hipGetErrorString(e);
    airebo_ctx_free(c);
    return fail(AIREBO_E_DEVICE, "context setup: " + m);
  }
  *out = c;
  return 0;
}

}  // namespace

extern "C" {

int airebo_params_load(const char* path, airebo_params_t* out) {
  if (!path || !out) return fail(AIREBO_E_ARG, "null argument");
  auto* s = new airebo_params_set();
  s->tri.resize((size_t)TRI_N * kTriCells * kTriCoef);
  std::string err;
  if (!build_params(path, s->P, s->tri.data(), err)) { delete s; return fail(AIREBO_E_PARAMS, err); }
  *out = s;
  return 0;
}

int airebo_params_parse(const char* text, size_t len, airebo_params_t* out) {
  if (!text || !out) return fail(AIREBO_E_ARG, "null argument");
  auto* s = new airebo_params_set();
  s->tri.resize((size_t)TRI_N * kTriCells * kTriCoef);
  std::string err;
  if (!build_params_text(text, len, s->P, s->tri.data(), err)) { delete s; return fail(AIREBO_E_PARAMS, err); }
  *out = s;
  return 0;
}

void airebo_params_free(airebo_params_t params) { delete params; }

int airebo_ctx_create_from_params(airebo_params_t params, const airebo_options* opt, airebo_ctx_t* out) {
  if (!params || !out) return fail(AIREBO_E_ARG, "null argument");
  airebo_options o;
  if (opt) o = *opt; else airebo_options_default(&o);
  int rc = check_options(o);
  if (rc) return rc;
  return ctx_create_impl(params->P, params->tri, o, out);
}

int airebo_ctx_create(const char* path, const airebo_options* opt, airebo_ctx_t* out) {
  if (!path || !out) return fail(AIREBO_E_ARG, "null argument");
  airebo_options o;
  if (opt) o = *opt; else airebo_options_default(&o);
  int rc = check_options(o);
  if (rc) return rc;
  airebo_params_t s = nullptr;
  rc = airebo_params_load(path, &s);
  if (rc) return rc;
  rc = ctx_create_impl(s->P, s->tri, o, out);
  airebo_params_free(s);
  return rc;
}

void airebo_ctx_free(airebo_ctx_t c) {
  if (!c) return;
  if (c->md.exec) (void)hipGraphExecDestroy(c->md.exec);
  if (c->md.graph) (void)hipGraphDestroy(c->md.graph);
  if (c->md.cs) (void)hipStreamDestroy(c->md.cs);
  void* mdp[] = {c->md.vel, c->md.xsave, c->md.vsave, c->md.ssave, c->md.ctl, c->md.scratch};
  for (void* p : mdp)
    if (p) hipFree(p);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  void* ptrs[] = {c->dP, c->dtri, c->x, c->xref, c->xsort, c->cell_of, c->cell_count, c->cell_start, c->cell_cursor,
                  c->cell_atoms, c->lj_n, c->lj_e, c->lf_n, c->lf_e, c->in_n, c->in_e, c->sn, c->sj, c->sd, c->sw, c->NCt, c->NHt,
                  c->bcount, c->bonds, c->qcount, c->q, c->F, c->F32, c->acc, c->dsys, c->atom_sys, c->sys_acc,
                  c->stats, c->flags, c->step, c->hx, c->hs};
  for (void* p : ptrs)
    if (p) hipFree(p);
  delete c;
}

}  // extern "C"

namespace {

// Size buffers for a batch of nsys systems (atoms of system k are
// [off[k], off[k+1]); box and periodic flags [nsys][3]); fill the Dev
// descriptor and upload the per-system boxes.
void md_end_impl(airebo_ctx* c);

// Boxes and cell grids of a batch (atoms of system k are [off[k], off[k+1]));
// box lengths and periodic flags [nsys][3].  A periodic side must hold the
// LJ list cutoff and twice the reach of a three-bond path (so that a path
// map keyed by atom index meets one image of each atom only).
int plan_boxes(const airebo_ctx* c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers,
               std::vector<SysBox>& hsys, size_t& ncell) {
  if (nsys < 1 || !off || !boxes || !pers) return fail(AIREBO_E_ARG, "null box, periodic or offsets");
  int64_t n = off[nsys] - off[0];
  if (off[0] != 0 || n < 0 || n >= (1ll << 27)) return fail(AIREBO_E_ARG, "n out of range");
  const DevParams& P = c->P;
  double rlist = P.rc_max + c->opt.skin;
  double lmin = std::max(2.0 * P.r_conn, rlist);
  hsys.resize(nsys);
  ncell = 0;
  for (int k = 0; k < nsys; ++k) {
    if (off[k + 1] < off[k]) return fail(AIREBO_E_ARG, "system offsets must not decrease");
    SysBox& B = hsys[k];
    std::memset(&B, 0, sizeof B);
    size_t nc_k = 1;
    for (int d = 0; d < 3; ++d) {
      double L = boxes[3 * k + d];
      if (!(L > 0) || !std::isfinite(L)) return fail(AIREBO_E_BOX, "box lengths must be positive");
      B.L[d] = L;
      B.invL[d] = 1.0 / L;
      B.per[d] = pers[3 * k + d] ? 1 : 0;
      if (B.per[d] && L < lmin)
        return fail(AIREBO_E_BOX, "periodic box side must be at least max(6 max R2, LJ cutoff + skin) = " +
                                      std::to_string(lmin) + " A");
      B.nc[d] = std::min(std::max(1, (int)std::floor(L / (0.5 * rlist))), 1024);   // cells >= half the list cutoff
      nc_k *= B.nc[d];
    }
    B.cell_off = (int)ncell;
    B.natoms = (int)(off[k + 1] - off[k]);
    ncell += nc_k;
  }
  return 0;
}

// Whether every periodic side holds twice the LJ list cutoff plus twice the
// skin (listed pairs never reach half a side before the next build).
int minimum_image_ok(const airebo_ctx* c, const std::vector<SysBox>& hsys) {
  double need = 2.0 * (c->P.rc_max + 2.0 * c->opt.skin);
  for (const SysBox& B : hsys)
    for (int d = 0; d < 3; ++d)
      if (B.per[d] && B.L[d] < need) return 0;
  return 1;
}

int setup(airebo_ctx* c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers, hipStream_t s,
          bool keep_md = false) {
  // any other use of the context ends an MD session: its captured step holds the buffers set up here
  if (c->md.on && !keep_md) md_end_impl(c);
  size_t ncell = 0;
  int prc = plan_boxes(c, nsys, off, boxes, pers, c->hsys, ncell);
  if (prc) return prc;
  int64_t n = off[nsys] - off[0];
  const DevParams& P = c->P;
  Dev& D = c->D;
  std::memset(&D, 0, sizeof D);
  D.n = (int)n;
  D.nsys = nsys;
  D.skin = c->opt.skin;
  c->hatom_sys.clear();
  c->ncell = (int)ncell;
  for (int p = 0; p < 3; ++p) {
    D.rlist2[p] = (P.rc[p] + c->opt.skin) * (P.rc[p] + c->opt.skin);
    D.rint2[p] = (P.R2[p] + c->opt.skin) * (P.R2[p] + c->opt.skin);
  }
  if (c->lj_cap == 0) c->lj_cap = c->opt.lj_cap > 0 ? c->opt.lj_cap : 160;
  if (c->lf_cap == 0) c->lf_cap = c->opt.lj_cap > 0 ? c->opt.lj_cap : 320;
  size_t N = (size_t)std::max<int64_t>(n, 1);
  int rc = 0;
  rc |= grow(c->x, c->cx, N);
  rc |= grow(c->xref, c->cxr, N);
  rc |= grow(c->xsort, c->cxs, N);
  rc |= grow(c->cell_of, c->c_of, N);
  rc |= grow(c->cell_count, c->c_cc, ncell);
  rc |= grow(c->cell_start, c->c_cs, ncell + 1);
  rc |= grow(c->cell_cursor, c->c_cu, ncell);
  rc |= grow(c->cell_atoms, c->c_ca, N);
  rc |= grow(c->lj_n, c->c_ljn, N);
  rc |= grow(c->lj_e, c->c_lje, N * (size_t)c->lj_cap);
  rc |= grow(c->lf_n, c->c_lfn, N);
  rc |= grow(c->lf_e, c->c_lfe, N * (size_t)c->lf_cap);
  rc |= grow(c->in_n, c->c_inn, N);
  rc |= grow(c->in_e, c->c_ine, N * c->icap);
  rc |= grow(c->sn, c->c_sn, N);
  rc |= grow(c->sj, c->c_sj, N * c->scap);
  rc |= grow(c->sd, c->c_sd, N * c->scap);
  rc |= grow(c->sw, c->c_sw, N * c->scap);
  rc |= grow(c->NCt, c->c_nc, N);
  rc |= grow(c->NHt, c->c_nh, N);
  rc |= grow(c->bcount, c->c_bc, 4);
  size_t bcap = N * c->scap / 2 + 64;
  rc |= grow(c->bonds, c->c_b, 3 * bcap);
  rc |= grow(c->qcount, c->c_qc, NSEG * QSTRIDE);
  size_t qcap = ((size_t)c->q_per_atom * N + 1024 * NSEG) / NSEG;   // per segment
  rc |= grow(c->q, c->c_q, qcap * NSEG);
  rc |= grow(c->F, c->c_F, 3 * N);
  if (c->opt.precision == AIREBO_SINGLE) {
    size_t had = c->c_F32;
    rc |= grow(c->F32, c->c_F32, 3 * N);
    // the FP32 sums start at zero; every evaluation leaves them at zero
    if (!rc && c->c_F32 != had && hipMemsetAsync(c->F32, 0, c->c_F32 * sizeof(float), s) != hipSuccess)
      rc |= fail(AIREBO_E_DEVICE, "clearing the FP32 force sums failed");
  }
  rc |= grow(c->acc, c->c_acc, NSLOT * A_N);
  rc |= grow(c->stats, c->c_st, S_N);
  rc |= grow(c->flags, c->c_fl, 4);
  {
    size_t had = c->c_stp;
    rc |= grow(c->step, c->c_stp, 4);
    // step counter and the last-block counters start at zero
    if (!rc && c->c_stp != had && hipMemsetAsync(c->step, 0, 4 * sizeof(int), s) != hipSuccess)
      rc |= fail(AIREBO_E_DEVICE, "clearing the step counters failed");
  }
  rc |= grow(c->dsys, c->c_dsys, nsys);
  if (nsys > 1) {
    rc |= grow(c->atom_sys, c->c_asys, N);
    rc |= grow(c->sys_acc, c->c_sacc, (size_t)nsys * A_N);
  }
  if (rc) return AIREBO_E_DEVICE;
  HIPCHK(hipMemcpyAsync(c->dsys, c->hsys.data(), sizeof(SysBox) * nsys, hipMemcpyHostToDevice, s));
  if (nsys > 1) {
    c->hatom_sys.resize(n);
    for (int k = 0; k < nsys; ++k)
      for (int64_t i = off[k]; i < off[k + 1]; ++i) c->hatom_sys[i] = k;
    HIPCHK(hipMemcpyAsync(c->atom_sys, c->hatom_sys.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  }
  D.sys = c->dsys;
  D.atom_sys = nsys > 1 ? c->atom_sys : nullptr;
  D.sys_acc = nsys > 1 ? c->sys_acc : nullptr;
  D.x = c->x; D.xref = c->xref; D.xsort = c->xsort; D.cell_of = c->cell_of; D.cell_count = c->cell_count; D.cell_start = c->cell_start;
  D.cell_cursor = c->cell_cursor; D.cell_atoms = c->cell_atoms; D.lj_cap = c->lj_cap; D.lj_n = c->lj_n;
  D.lj_e = c->lj_e; D.lf_cap = c->lf_cap; D.lf_n = c->lf_n; D.lf_e = c->lf_e; D.in_n = c->in_n;
  D.rnear = P.r_conn + c->opt.skin;
  D.minimg = minimum_image_ok(c, c->hsys); D.in_e = c->in_e; D.sn = c->sn; D.sj = c->sj; D.sd = c->sd; D.sw = c->sw;
  D.icap = c->icap;
  D.scap = c->scap;
  D.slog2 = 31 - __builtin_clz((unsigned)c->scap);
  D.NCt = c->NCt; D.NHt = c->NHt; D.bcap = (int)bcap; D.bcount = c->bcount; D.bonds = c->bonds;
  D.qcap = (int)qcap; D.qcount = c->qcount;
  D.q = c->q; D.F = c->F; D.F32 = c->F32; D.acc = c->acc; D.stats = c->stats; D.flags = c->flags; D.step = c->step;
  return 0;
}

inline int blocks(int64_t n, int t) { return (int)std::max<int64_t>(1, (n + t - 1) / t); }

// Launch the rebuild chain (kernels check the rebuild flag on the device).
void launch_rebuild(airebo_ctx* c, hipStream_t s) {
  Dev& D = c->D;
  int ncell = c->ncell;
  LAUNCH(c, K_BIN, k_bin, dim3(blocks(D.n, 1024)), dim3(1024), s, D, ncell);   // last block scans the counts
  LAUNCH(c, K_FILL, k_fill, dim3(blocks(D.n, 256)), dim3(256), s, D);
  LAUNCH(c, K_BUILD, k_build, dim3(blocks((int64_t)D.n * WAVE, 256)), dim3(256), s, D, (const DevParams*)c->dP);
}

// Launch one force evaluation on the current positions.
// zero = false when the step's k_kick_drift has already zeroed the forces and
// accumulators.
void launch_forces(airebo_ctx* c, hipStream_t s, bool zero = true) {
  Dev& D = c->D;
  const DevParams* P = c->dP;
  int mask = c->opt.term_mask;
  if (zero) LAUNCH(c, K_ZERO, k_zero,
         dim3(std::min(std::max({blocks(3 * (int64_t)D.n, 256), NSLOT * A_N / 256, blocks((int64_t)D.nsys * A_N, 256)}),
                       4096)),
         dim3(256), s, D);
  int sblk = c->opt.short_block ? c->opt.short_block : 1024;
  const int prec = c->opt.precision;
  const bool single = prec == AIREBO_SINGLE;
  int bblk = c->opt.bond_block ? c->opt.bond_block : 64;
  int nb = c->opt.bond_grid ? c->opt.bond_grid : std::min(blocks((int64_t)D.n * 2, bblk), 8192);
  int qblk = c->opt.defer_block ? c->opt.defer_block : 64;
  const bool bonded = mask & (AIREBO_TERM_REBO | AIREBO_TERM_TORSION);
  const bool lj = mask & AIREBO_TERM_LJ;
  // arithmetic type R, accumulation type A: FP64 (double, double), mixed
  // (float, double), single (float, float)
  const bool morse = c->opt.vdw == AIREBO_VDW_MORSE;   // FP64 only (checked at context creation)
  auto far_pairs = [&](hipStream_t st) {
    dim3 glf(blocks((int64_t)D.n * LJF_G, 256));
    if (D.minimg) {
      if (morse) LAUNCH(c, K_LJF, (k_ljf<double, double, true, true>), glf, dim3(256), st, D, P);
      else if (prec == AIREBO_MIXED) LAUNCH(c, K_LJF, (k_ljf<float, double, false, true>), glf, dim3(256), st, D, P);
      else if (single) LAUNCH(c, K_LJF, (k_ljf<float, float, false, true>), glf, dim3(256), st, D, P);
      else LAUNCH(c, K_LJF, (k_ljf<double, double, false, true>), glf, dim3(256), st, D, P);
    } else {
      if (morse) LAUNCH(c, K_LJF, (k_ljf<double, double, true, false>), glf, dim3(256), st, D, P);
      else if (prec == AIREBO_MIXED) LAUNCH(c, K_LJF, (k_ljf<float, double, false, false>), glf, dim3(256), st, D, P);
      else if (single) LAUNCH(c, K_LJF, (k_ljf<float, float, false, false>), glf, dim3(256), st, D, P);
      else LAUNCH(c, K_LJF, (k_ljf<double, double, false, false>), glf, dim3(256), st, D, P);
    }
  };
  auto short_list = [&](hipStream_t st) {   // SHORT_G lanes per atom
    if (single) LAUNCH(c, K_SHORT, k_short<true>, dim3(blocks((int64_t)D.n * SHORT_G, sblk)), dim3(sblk), st, D, P);
    else LAUNCH(c, K_SHORT, k_short<false>, dim3(blocks((int64_t)D.n * SHORT_G, sblk)), dim3(sblk), st, D, P);
  };
  auto near_pairs = [&](hipStream_t st) {
    dim3 glj(blocks((int64_t)D.n * WAVE, LJ_BLOCK));
    if (morse) LAUNCH(c, K_LJ, (k_lj<double, double, true>), glj, dim3(LJ_BLOCK), st, D, P);
    else if (prec == AIREBO_MIXED) LAUNCH(c, K_LJ, (k_lj<float, double, false>), glj, dim3(LJ_BLOCK), st, D, P);
    else if (single) LAUNCH(c, K_LJ, (k_lj<float, float, false>), glj, dim3(LJ_BLOCK), st, D, P);
    else LAUNCH(c, K_LJ, (k_lj<double, double, false>), glj, dim3(LJ_BLOCK), st, D, P);
  };
  // the bond-order kernels stage each lane's neighbourhood in LDS (dynamic size)
  const size_t sh32 = (size_t)stage_bytes<float>(), sh64 = (size_t)stage_bytes<double>();
  auto bond_terms = [&](hipStream_t st) {
    if (prec == AIREBO_MIXED)
      LAUNCH_SHM(c, K_BOND, (k_bond<float, double>), dim3(nb), dim3(bblk), bblk * sh32, st, D, P, mask);
    else if (single) LAUNCH_SHM(c, K_BOND, (k_bond<float, float>), dim3(nb), dim3(bblk), bblk * sh32, st, D, P, mask);
    else LAUNCH_SHM(c, K_BOND, (k_bond<double, double>), dim3(nb), dim3(bblk), bblk * sh64, st, D, P, mask);
  };
  auto deferred_pairs = [&](hipStream_t st) {
    // one lane per expected deferred pair (about 3 per atom in dense melts), so
    // that the latency-bound b* work is spread over many wavefronts
    dim3 gq(std::min(blocks(4 * (int64_t)D.n, qblk), 16384));
    if (morse) LAUNCH_SHM(c, K_BSTAR, (k_bstar<double, double, true>), gq, dim3(qblk), qblk * sh64, st, D, P);
    else if (prec == AIREBO_MIXED)
      LAUNCH_SHM(c, K_BSTAR, (k_bstar<float, double, false>), gq, dim3(qblk), qblk * sh32, st, D, P);
    else if (single) LAUNCH_SHM(c, K_BSTAR, (k_bstar<float, float, false>), gq, dim3(qblk), qblk * sh32, st, D, P);
    else LAUNCH_SHM(c, K_BSTAR, (k_bstar<double, double, false>), gq, dim3(qblk), qblk * sh64, st, D, P);
  };
  // Two streams.  The main stream runs the short list, the near LJ pairs
  // (they need the short list for the path maps) and the deferred pairs; the
  // second runs the far LJ pairs and the bonded terms, forked either after
  // the short list (far pairs beside the near pairs, then the bonded terms
  // beside the deferred pairs) or after the near pairs (bonded terms, then
  // far pairs, both beside the deferred pairs).  Measured: in FP64 from about
  // 5 x 10^4 atoms the two FP64 pair kernels side by side compete for the
  // vector units and the second order is 1-2.5% faster; in mixed and single
  // precision, for small systems and for batches of small systems (whose
  // bonded and deferred work is latency-bound) the first is faster, by up to
  // 13% on batches.  (The profiler's per-kernel events keep everything on one
  // stream.)
  const bool two = !c->prof && lj && bonded;
  int sched = c->opt.schedule;
  if (sched == AIREBO_SCHED_AUTO)
    sched = prec == AIREBO_FP64 && D.nsys == 1 && D.n > AIREBO_SCHED_AUTO_ATOMS ? AIREBO_SCHED_FAR_AFTER_NEAR
                                                                              : AIREBO_SCHED_FAR_WITH_NEAR;
  if (!two) {
    short_list(s);
    if (lj) { near_pairs(s); far_pairs(s); }
    if (bonded) bond_terms(s);
    if (lj) deferred_pairs(s);
  } else if (sched == AIREBO_SCHED_FAR_WITH_NEAR) {
    short_list(s);
    (void)hipEventRecord(c->ev_fork, s);
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    far_pairs(c->side);
    bond_terms(c->side);
    near_pairs(s);
    deferred_pairs(s);
  } else {
    short_list(s);
    near_pairs(s);
    (void)hipEventRecord(c->ev_fork, s);
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    bond_terms(c->side);
    far_pairs(c->side);
    deferred_pairs(s);
  }
  if (two) {
    (void)hipEventRecord(c->ev_join, c->side);
    (void)hipStreamWaitEvent(s, c->ev_join, 0);
  }
  if (single) LAUNCH(c, K_FOLD32, k_fold32, dim3(std::min(blocks(3 * (int64_t)D.n, 256), 4096)), dim3(256), s, D);
}

int check_flags(airebo_ctx* c, int flags) {
  if (flags & F_BADSPEC) return fail(AIREBO_E_SPECIES, "species codes must be 0 (C) or 1 (H)");
  if (flags & F_NONFINITE) return fail(AIREBO_E_NONFINITE, "non-finite position or energy");
  if (flags & F_OV_SHORT)
    return fail(AIREBO_E_CAPACITY, "an atom has more than " + std::to_string(c->scap) + " REBO neighbours");
  if (flags & F_OV_INT)
    return fail(AIREBO_E_CAPACITY, "an atom has more than " + std::to_string(c->icap) +
                                       " atoms within the REBO cutoff plus skin");
  if (flags & F_OV_PATH) return fail(AIREBO_E_CAPACITY, "path map capacity exceeded");
  if (flags & F_OV_BOND) return fail(AIREBO_E_CAPACITY, "bond list capacity exceeded");
  if (flags & F_OV_QUEUE) return fail(AIREBO_E_CAPACITY, "b* queue capacity exceeded");
  if (flags & F_OV_LJ) return fail(AIREBO_E_CAPACITY, "LJ list capacity exceeded");
  if (flags & F_OV_NN) return fail(AIREBO_E_CAPACITY, "more than 192 neighbours within 6 A or 48 within 3.5 A");
  return 0;
}

// Capacities that grow when an evaluation or MD chunk overflows them.
constexpr int F_GROW = F_OV_LJ | F_OV_QUEUE | F_OV_SHORT | F_OV_INT;

// Capacity growth after an overflow reported in `flags`: the short and
// intermediate lists to twice their entries per atom, the LJ list to the
// largest row seen (plus headroom), the deferred-pair queue to twice its
// entries per atom.  Returns nonzero when a limit is reached.
int grow_caps(airebo_ctx* c, int flags) {
  ++c->regrow;
  if (flags & F_OV_SHORT) {
    if (c->scap >= SCAP_MAX) return 1;
    c->scap *= 2;
  }
  if (flags & F_OV_INT) {
    if (c->icap >= ICAP_MAX) return 1;
    c->icap = std::min(2 * c->icap, ICAP_MAX);
  }
  if (flags & F_OV_LJ) {   // both parts of the LJ list
    if (c->lj_cap >= (1 << 16) && c->lf_cap >= (1 << 16)) return 1;
    auto up = [](int cap, unsigned long long mx) {
      unsigned long long need = mx + mx / 4 + 32;
      return (int)std::min<unsigned long long>(std::max<unsigned long long>(need, cap + cap / 2 + 32), 1u << 16);
    };
    c->lj_cap = up(c->lj_cap, c->host_stats[S_MAXLJ]);
    c->lf_cap = up(c->lf_cap, c->host_stats[S_MAXLF]);
  }
  if (flags & F_OV_QUEUE) {
    if (c->q_per_atom >= 1024) return 1;
    c->q_per_atom *= 2;
  }
  return 0;
}

// One evaluation of a batch; forces == nullptr evaluates into the context's
// own buffer.  energy [nsys][4], virial [nsys][6] (device).
int compute_impl(airebo_ctx_t c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers,
                 const double* pos, const int32_t* species, double* energy, double* forces, double* virial,
                 void* stream) {
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(c->opt.device));
  c->regrow = 0;
  for (int attempt = 0; attempt < 6; ++attempt) {
    int rc = setup(c, nsys, off, boxes, pers, s);
    if (rc) return rc;
    Dev& D = c->D;
    int64_t n = D.n;
    D.F = forces ? forces : c->F;
    HIPCHK(hipMemsetAsync(c->stats, 0, S_N * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, D, F_REBUILD);
    HIPCHK(hipMemsetAsync(c->cell_count, 0, sizeof(int) * c->ncell, s));
    if (n > 0) {
      hipLaunchKernelGGL(k_load, dim3(blocks(n, 256)), dim3(256), 0, s, D, pos, species, 0);
      launch_rebuild(c, s);
      launch_forces(c, s);
    } else {
      hipLaunchKernelGGL(k_zero, dim3(std::max(NSLOT * A_N / 256, blocks((int64_t)nsys * A_N, 256))), dim3(256), 0,
                         s, D);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, D, energy, virial);
    if (n > 0) {
      int g = std::min(blocks(n, 256), 1024);
      hipLaunchKernelGGL(k_max, dim3(g), dim3(256), 0, s, (const int*)D.lj_n, (int)n, D.lj_cap, D.stats + S_MAXLJ,
                         D.stats + S_LJENT, (unsigned long long*)nullptr);
      hipLaunchKernelGGL(k_max, dim3(g), dim3(256), 0, s, (const int*)D.lf_n, (int)n, D.lf_cap, D.stats + S_MAXLF,
                         D.stats + S_LJENT, D.stats + S_LFENT);
    }
    HIPCHK(hipGetLastError());
    int flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->host_stats, c->stats, sizeof c->host_stats, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    c->host_stats[S_REGROW] = c->regrow;
    if ((flags & F_GROW) && !(flags & (F_BADSPEC | F_NONFINITE))) {   // grow what overflowed and evaluate again
      if (grow_caps(c, flags)) return check_flags(c, flags);
      continue;
    }
    return check_flags(c, flags);
  }
  return fail(AIREBO_E_CAPACITY, "list or queue capacities could not be established");
}

// One evaluation with every work buffer in the device's static work area
// (no allocation).  The context lends its parameters, streams and events;
// its own buffers and state are left as they were.
int compute_static_impl(airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species, const double* box,
                        const int32_t* periodic, double* energy, double* forces, double* virial, hipStream_t s) {
  if (n > STATIC_MAX_ATOMS)
    return fail(AIREBO_E_CAPACITY, "airebo_compute_static takes at most " + std::to_string(STATIC_MAX_ATOMS) +
                                       " atoms (" + std::to_string(n) + " given)");
  int dev = c->opt.device;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    base = static_cast<unsigned char*>(g_static_ptr[dev]);
  }
  if (!base) return fail(AIREBO_E_DEVICE, "static work area of this device not initialised");
  HIPCHK(hipSetDevice(dev));
  if (c->md.on) md_end_impl(c);
  int64_t off[2] = {0, n};
  std::vector<SysBox> hsys;
  size_t ncell = 0;
  int rc = plan_boxes(c, 1, off, box, periodic, hsys, ncell);
  if (rc) return rc;
  if (ncell > (size_t)STATIC_MAX_CELLS)
    return fail(AIREBO_E_CAPACITY, "cell grid of " + std::to_string(ncell) + " cells exceeds the static limit of " +
                                       std::to_string(STATIC_MAX_CELLS));
  const DevParams& P = c->P;
  Dev saved = c->D;
  int saved_ncell = c->ncell;
  Dev& D = c->D;
  std::memset(&D, 0, sizeof D);
  const StaticLayout& L = kStatic;
  D.n = (int)n;
  D.nsys = 1;
  D.skin = c->opt.skin;
  for (int p = 0; p < 3; ++p) {
    D.rlist2[p] = (P.rc[p] + c->opt.skin) * (P.rc[p] + c->opt.skin);
    D.rint2[p] = (P.R2[p] + c->opt.skin) * (P.R2[p] + c->opt.skin);
  }
  D.sys = reinterpret_cast<SysBox*>(base + L.sys);
  D.x = reinterpret_cast<double4*>(base + L.x);
  D.xref = reinterpret_cast<double4*>(base + L.xref);
  D.xsort = reinterpret_cast<float4*>(base + L.xsort);
  D.cell_of = reinterpret_cast<int*>(base + L.cell_of);
  D.cell_count = reinterpret_cast<int*>(base + L.cell_count);
  D.cell_start = reinterpret_cast<int*>(base + L.cell_start);
  D.cell_cursor = reinterpret_cast<int*>(base + L.cell_cursor);
  D.cell_atoms = reinterpret_cast<int*>(base + L.cell_atoms);
  D.lj_n = reinterpret_cast<int*>(base + L.lj_n);
  D.lj_e = reinterpret_cast<unsigned*>(base + L.lj_e);
  D.lf_n = reinterpret_cast<int*>(base + L.lf_n);
  D.lf_e = reinterpret_cast<unsigned*>(base + L.lf_e);
  D.rnear = P.r_conn + c->opt.skin;
  D.minimg = minimum_image_ok(c, hsys);
  D.in_n = reinterpret_cast<int*>(base + L.in_n);
  D.in_e = reinterpret_cast<int*>(base + L.in_e);
  D.icap = ICAP;
  D.scap = SCAP;
  D.slog2 = 3;
  static_assert(SCAP == 8, "static short-list stride");
  D.sn = reinterpret_cast<int*>(base + L.sn);
  D.sj = reinterpret_cast<int*>(base + L.sj);
  D.sd = reinterpret_cast<double4*>(base + L.sd);
  D.sw = reinterpret_cast<double2*>(base + L.sw);
  D.NCt = reinterpret_cast<double*>(base + L.NCt);
  D.NHt = reinterpret_cast<double*>(base + L.NHt);
  D.bcount = reinterpret_cast<int*>(base + L.bcount);
  D.bonds = reinterpret_cast<int2*>(base + L.bonds);
  D.bcap = (int)(std::max<int64_t>(n, 1) * SCAP / 2 + 64);
  D.qcount = reinterpret_cast<int*>(base + L.qcount);
  D.q = reinterpret_cast<int4*>(base + L.q);
  D.qcap = (int)(STATIC_QUEUE / NSEG);
  D.F = forces;
  D.F32 = c->opt.precision == AIREBO_SINGLE ? reinterpret_cast<float*>(base + L.F32) : nullptr;
  D.acc = reinterpret_cast<double*>(base + L.acc);
  D.stats = reinterpret_cast<unsigned long long*>(base + L.stats);
  D.flags = reinterpret_cast<int*>(base + L.flags);
  D.step = reinterpret_cast<int*>(base + L.step);
  c->ncell = (int)ncell;
  const int64_t nn = std::max<int64_t>(n, 1);
  D.lj_cap = (int)std::min<int64_t>(160, STATIC_LJ_ENTRIES / nn);
  D.lf_cap = (int)std::min<int64_t>(320, STATIC_LF_ENTRIES / nn);
  auto done = [&](int code) {
    c->D = saved;
    c->ncell = saved_ncell;
    return code;
  };
  hipLaunchKernelGGL(k_put_box, dim3(1), dim3(64), 0, s, reinterpret_cast<SysBox*>(base + L.sys), hsys[0]);
  // the FP32 force sums of single precision start at zero (the array keeps
  // whatever the last call on this device left)
  if (D.F32 && n > 0) {
    hipError_t e = hipMemsetAsync(D.F32, 0, sizeof(float) * 3 * n, s);
    if (e != hipSuccess) return done(fail(AIREBO_E_DEVICE, std::string("clearing FP32 sums: ") + hipGetErrorString(e)));
  }
  for (int attempt = 0; attempt < 3; ++attempt) {
    hipError_t e = hipMemsetAsync(D.stats, 0, S_N * sizeof(unsigned long long), s);
    if (e == hipSuccess) e = hipMemsetAsync(D.cell_count, 0, sizeof(int) * ncell, s);
    if (e == hipSuccess) e = hipMemsetAsync(D.step, 0, 4 * sizeof(int), s);   // step and last-block counters
    if (e != hipSuccess) return done(fail(AIREBO_E_DEVICE, std::string("static clear: ") + hipGetErrorString(e)));
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, D, F_REBUILD);
    if (n > 0) {
      hipLaunchKernelGGL(k_load, dim3(blocks(n, 256)), dim3(256), 0, s, D, pos, species, 0);
      launch_rebuild(c, s);
      launch_forces(c, s);
    } else {
      hipLaunchKernelGGL(k_zero, dim3(NSLOT * A_N / 256), dim3(256), 0, s, D);
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, D, energy, virial);
    if (n > 0) {
      hipLaunchKernelGGL(k_max, dim3(std::min(blocks(n, 256), 1024)), dim3(256), 0, s, (const int*)D.lj_n, (int)n,
                         D.lj_cap, D.stats + S_MAXLJ, D.stats + S_LJENT, (unsigned long long*)nullptr);
      hipLaunchKernelGGL(k_max, dim3(std::min(blocks(n, 256), 1024)), dim3(256), 0, s, (const int*)D.lf_n, (int)n,
                         D.lf_cap, D.stats + S_MAXLF, D.stats + S_LJENT, D.stats + S_LFENT);
    }
    int flags = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&flags, D.flags, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->host_stats, D.stats, sizeof c->host_stats, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return done(fail(AIREBO_E_DEVICE, std::string("static evaluation: ") + hipGetErrorString(e)));
    c->host_stats[S_REGROW] = (unsigned long long)attempt;
    if (flags & F_OV_LJ) {   // longer LJ rows, if the area holds them
      int64_t need = (int64_t)c->host_stats[S_MAXLJ] + 32, needf = (int64_t)c->host_stats[S_MAXLF] + 32;
      if (need * nn > STATIC_LJ_ENTRIES || needf * nn > STATIC_LF_ENTRIES)
        return done(fail(AIREBO_E_CAPACITY, "LJ list of " + std::to_string(need) + " near and " +
                                                std::to_string(needf) + " far entries per atom exceeds the static "
                                                "work area"));
      D.lj_cap = (int)need;
      D.lf_cap = (int)needf;
      continue;
    }
    if (flags & F_OV_QUEUE) return done(fail(AIREBO_E_CAPACITY, "deferred-pair queue exceeds the static work area"));
    if (flags & (F_OV_SHORT | F_OV_INT))
      return done(fail(AIREBO_E_CAPACITY, "more than 8 short or 48 intermediate neighbours of an atom exceed the "
                                          "static work area"));
    return done(check_flags(c, flags));
  }
  return done(fail(AIREBO_E_CAPACITY, "LJ list capacity could not be established in the static work area"));
}

// ---------------------------------------------------------------------------
// Molecular dynamics: velocity Verlet (Sec. 2) in a session held by the
// context.  md_begin loads positions and velocities, sizes the lists with one
// evaluation, computes the initial forces and captures one step into a HIP
// graph; md_run replays it in chunks; md_state copies the state out.
// Before each chunk the state (positions, velocities, statistics, step
// counter) is copied aside on the device.  After the chunk every error flag
// is read: a list or queue overflow restores the state, grows the capacity,
// recomputes the forces of the restored state and captures the step again;
// a non-finite step restores the state and returns the error.
// ---------------------------------------------------------------------------
constexpr int64_t MD_CHUNK = 256;
constexpr int F_ERRORS = F_OV_SHORT | F_OV_INT | F_OV_LJ | F_OV_PATH | F_OV_BOND | F_OV_QUEUE | F_NONFINITE |
                         F_BADSPEC | F_OV_NN;

void md_release_graph(airebo_ctx* c) {
  if (c->md.exec) (void)hipGraphExecDestroy(c->md.exec);
  if (c->md.graph) (void)hipGraphDestroy(c->md.graph);
  c->md.exec = nullptr;
  c->md.graph = nullptr;
}

void md_end_impl(airebo_ctx* c) {
  md_release_graph(c);
  c->md.on = false;
  c->md.forces = nullptr;
  c->md.skip = nullptr;
  c->D.skip = nullptr;
}

inline int thermo_block(int nsys) { return std::min(1024, std::max(64, ((nsys + 63) / 64) * 64)); }

// One step: thermo row of the previous state, kick and drift, rebuild when
// flagged, forces, kick.
void md_step(airebo_ctx* c, hipStream_t s) {
  Dev& D = c->D;
  int64_t n = D.n;
  auto& md = c->md;
  double half_skin2 = 0.25 * c->opt.skin * c->opt.skin;
  LAUNCH(c, K_KICK_DRIFT, k_kick_drift, dim3(blocks(n, 256)), dim3(256), s, D, md.vel, md.m0, md.m1, md.dt, half_skin2,
         (const MdCtl*)md.ctl);
  launch_rebuild(c, s);
  md.forces(s, false);
  LAUNCH(c, K_KICK, k_kick, dim3(blocks(n, 256)), dim3(256), s, D, md.vel, md.m0, md.m1, md.dt);
}

// Forces and kinetic energy of the positions in the context (after a load or
// a restore), with the lists rebuilt; clears the flags.
void md_prime(airebo_ctx* c, hipStream_t s) {
  Dev& D = c->D;
  hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, D, F_REBUILD);
  (void)hipMemsetAsync(c->cell_count, 0, sizeof(int) * c->ncell, s);
  launch_rebuild(c, s);
  c->md.forces(s, true);
  hipLaunchKernelGGL(k_kick, dim3(blocks(D.n, 256)), dim3(256), 0, s, D, c->md.vel, c->md.m0, c->md.m1, 0.0);
}

// Buffers of the session for the current capacities; the Dev descriptor
// pointed at the context's force array.
int md_setup(airebo_ctx* c, hipStream_t s) {
  auto& md = c->md;
  int rc = setup(c, md.nsys, md.off.data(), md.boxes.data(), md.pers.data(), s, true);
  if (rc) return rc;
  Dev& D = c->D;
  D.F = c->F;
  D.skip = md.skip;
  size_t n = (size_t)std::max(D.n, 1);
  rc |= grow(md.vel, md.c_vel, 3 * n);
  rc |= grow(md.xsave, md.c_xs, n);
  rc |= grow(md.vsave, md.c_vs, 3 * n);
  rc |= grow(md.ssave, md.c_ss, S_N + 1);
  if (!md.ctl) HIPCHK(hipMalloc(&md.ctl, sizeof(MdCtl)));
  return rc ? AIREBO_E_DEVICE : 0;
}

hipError_t md_capture(airebo_ctx* c) {
  auto& md = c->md;
  md_release_graph(c);
  if (!md.cs) {
    hipError_t e = hipStreamCreateWithFlags(&md.cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamBeginCapture(md.cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  md_step(c, md.cs);
  e = hipStreamEndCapture(md.cs, &md.graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&md.exec, md.graph, nullptr, nullptr, 0);
  return e;
}

int md_sync_flags(airebo_ctx* c, hipStream_t s, int& flags) {
  flags = 0;
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(&flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->host_stats, c->stats, sizeof c->host_stats, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->host_stats[S_REGROW] = c->regrow;
  return 0;
}

// Start a session.  `size` runs one evaluation that establishes the list
// capacities; `forces` launches one force evaluation of the session.
int md_begin_impl(airebo_ctx* c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers,
                  const double* pos, const double* vel, const int32_t* species, const double* mass, double dt,
                  hipStream_t s, const std::function<int()>& size, std::function<void(hipStream_t, bool)> forces,
                  const int* skip) {
  HIPCHK(hipSetDevice(c->opt.device));
  if (c->md.on) md_end_impl(c);
  int64_t n = off[nsys] - off[0];
  if (n < 1) return fail(AIREBO_E_ARG, "an MD session needs at least one atom");
  int rc = size();
  if (rc) return rc;
  // room for list growth between rebuilds
  auto sized = [&](unsigned long long mx) {
    unsigned long long slack = c->opt.lj_slack > 0 ? (unsigned long long)c->opt.lj_slack : mx / 4 + 32;
    return (int)std::min<unsigned long long>(std::max<unsigned long long>(mx + slack, 1), 1u << 16);
  };
  c->lj_cap = sized(c->host_stats[S_MAXLJ]);
  c->lf_cap = sized(c->host_stats[S_MAXLF]);
  auto& md = c->md;
  md.nsys = nsys;
  md.off.assign(off, off + nsys + 1);
  md.boxes.assign(boxes, boxes + 3 * (size_t)nsys);
  md.pers.assign(pers, pers + 3 * (size_t)nsys);
  md.m0 = mass[0];
  md.m1 = mass[1];
  md.dt = dt;
  md.forces = std::move(forces);
  md.skip = skip;
  rc = md_setup(c, s);
  if (rc) { md_end_impl(c); return rc; }
  Dev& D = c->D;
  HIPCHK(hipMemcpyAsync(md.vel, vel, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(c->stats, 0, S_N * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_load, dim3(blocks(n, 256)), dim3(256), 0, s, D, pos, species, 0);
  md_prime(c, s);
  int flags = 0;
  rc = md_sync_flags(c, s, flags);
  if (!rc && (flags & F_ERRORS)) rc = check_flags(c, flags);
  if (!rc && !c->prof) {
    hipError_t e = md_capture(c);
    if (e != hipSuccess) rc = fail(AIREBO_E_DEVICE, std::string("md capture: ") + hipGetErrorString(e));
  }
  if (rc) { md_end_impl(c); return rc; }
  md.on = true;
  return 0;
}

// Advance the session by nsteps; thermo rows [nsteps / every + 1][nsys][7]
// (device; row 0 is the state at the start of the run).
int md_run_impl(airebo_ctx* c, int64_t nsteps, int64_t every, double* thermo, hipStream_t s) {
  auto& md = c->md;
  if (!md.on) return fail(AIREBO_E_ARG, "no MD session (airebo_md_begin)");
  HIPCHK(hipSetDevice(c->opt.device));
  Dev& D = c->D;
  int64_t n = D.n;
  MdCtl h{every > 0 ? thermo : nullptr, (int)std::max<int64_t>(every, 0),
          every > 0 ? (int)(nsteps / every) + 1 : 0};
  static_assert(sizeof(MdCtl) <= sizeof md.hctl, "control block image");
  std::memcpy(md.hctl, &h, sizeof h);
  HIPCHK(hipMemcpyAsync(md.ctl, md.hctl, sizeof(MdCtl), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(c->step, 0, sizeof(int), s));
  // Each step's first kernel writes the row of the state before it (row 0:
  // the current state, whose sums are those of the last evaluation); the
  // row of the final state is written after the last step.
  if (c->prof) {   // per-kernel timing: eager launches, one event pair per kernel
    HIPCHK(hipStreamSynchronize(s));
    for (auto& e : c->ev) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    c->ev.clear();
    for (int64_t k = 0; k < nsteps; ++k) md_step(c, s);
    hipLaunchKernelGGL(k_thermo, dim3(1), dim3(thermo_block(D.nsys)), 0, s, D, (const MdCtl*)md.ctl);
    int flags = 0;
    int rc = md_sync_flags(c, s, flags);
    if (rc) return rc;
    return (flags & F_ERRORS) ? check_flags(c, flags) : 0;
  }
  hipEvent_t ready = nullptr;   // the replays on the capture stream follow the caller's stream
  HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  (void)hipEventRecord(ready, s);
  (void)hipStreamWaitEvent(md.cs, ready, 0);
  (void)hipEventDestroy(ready);
  hipStream_t cs = md.cs;
  int regrow = 0;
  for (int64_t done = 0; done < nsteps;) {
    int64_t k = std::min(MD_CHUNK, nsteps - done);
    HIPCHK(hipMemcpyAsync(md.xsave, c->x, sizeof(double4) * n, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(md.vsave, md.vel, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(md.ssave, c->stats, sizeof(unsigned long long) * S_N, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(md.ssave + S_N, c->step, sizeof(int), hipMemcpyDeviceToDevice, cs));
    for (int64_t q = 0; q < k; ++q) HIPCHK(hipGraphLaunch(md.exec, cs));
    int flags = 0;
    int rc = md_sync_flags(c, cs, flags);
    if (rc) return rc;
    if (!(flags & F_ERRORS)) { done += k; continue; }
    // restore the state at the start of the chunk and recompute its forces
    HIPCHK(hipMemcpyAsync(c->x, md.xsave, sizeof(double4) * n, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(md.vel, md.vsave, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(c->stats, md.ssave, sizeof(unsigned long long) * S_N, hipMemcpyDeviceToDevice, cs));
    HIPCHK(hipMemcpyAsync(c->step, md.ssave + S_N, sizeof(int), hipMemcpyDeviceToDevice, cs));
    bool capacity = (flags & F_GROW) && !(flags & (F_ERRORS & ~F_GROW));
    if (capacity) {
      if (++regrow > 12 || grow_caps(c, flags)) {
        rc = check_flags(c, flags);
      } else {
        rc = md_setup(c, cs);
      }
    }
    md_prime(c, cs);
    int f2 = 0;
    int rc2 = md_sync_flags(c, cs, f2);
    if (rc) return rc;
    if (rc2) return rc2;
    if (!capacity) return check_flags(c, flags);
    if (f2 & F_ERRORS) return check_flags(c, f2);
    hipError_t e = md_capture(c);
    if (e != hipSuccess) return fail(AIREBO_E_DEVICE, std::string("md capture: ") + hipGetErrorString(e));
  }
  hipLaunchKernelGGL(k_thermo, dim3(1), dim3(thermo_block(D.nsys)), 0, cs, D, (const MdCtl*)md.ctl);
  HIPCHK(hipStreamSynchronize(cs));
  return 0;
}

// Current positions (wrapped into periodic boxes) and velocities.
int md_state_impl(airebo_ctx* c, double* pos, double* vel, hipStream_t s) {
  auto& md = c->md;
  if (!md.on) return fail(AIREBO_E_ARG, "no MD session (airebo_md_begin)");
  HIPCHK(hipSetDevice(c->opt.device));
  Dev& D = c->D;
  if (pos) hipLaunchKernelGGL(k_store, dim3(blocks(D.n, 256)), dim3(256), 0, s, D, pos);
  if (vel) HIPCHK(hipMemcpyAsync(vel, md.vel, sizeof(double) * 3 * D.n, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  return 0;
}

// Session of the AIREBO force field on a batch.
int md_begin_airebo(airebo_ctx* c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers,
                    const double* pos, const double* vel, const int32_t* species, const double* mass, double dt,
                    hipStream_t s) {
  auto size = [&]() -> int {
    size_t need = 10 * (size_t)nsys;
    if (grow(c->md.scratch, c->md.c_scr, need)) return AIREBO_E_DEVICE;
    return compute_impl(c, nsys, off, boxes, pers, pos, species, c->md.scratch, nullptr,
                        c->md.scratch + 4 * (size_t)nsys, s);
  };
  return md_begin_impl(c, nsys, off, boxes, pers, pos, vel, species, mass, dt, s, size,
                       [c](hipStream_t st, bool zero) { launch_forces(c, st, zero); }, nullptr);
}

// airebo_nve as one session: begin, run, state out, end.
int nve_impl(airebo_ctx_t c, int nsys, const int64_t* off, const double* boxes, const int32_t* pers, double* pos,
             double* vel, const int32_t* species, const double* mass, double dt, int64_t nsteps, int64_t every,
             double* thermo, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int64_t n = off[nsys] - off[0];
  if (n == 0) return 0;
  int rc = md_begin_airebo(c, nsys, off, boxes, pers, pos, vel, species, mass, dt, s);
  if (!rc) rc = md_run_impl(c, nsteps, every, thermo, s);
  // on an error the state is that of the last completed chunk
  int rc2 = c->md.on ? md_state_impl(c, pos, vel, s) : 0;
  if (c->md.on) {
    hipError_t e = hipStreamSynchronize(s);
    if (!rc2 && e != hipSuccess) rc2 = fail(AIREBO_E_DEVICE, std::string("nve: ") + hipGetErrorString(e));
  }
  md_end_impl(c);
  return rc ? rc : rc2;
}

}  // namespace

extern "C" {

int airebo_compute(airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species, const double* box,
                   const int32_t* periodic, double* energy, double* forces, double* virial, void* stream) {
  if (!c || (n > 0 && (!pos || !species || !forces)) || !energy || !virial || !box || !periodic)
    return fail(AIREBO_E_ARG, "null argument");
  if (n < 0) return fail(AIREBO_E_ARG, "n must be >= 0");
  int64_t off[2] = {0, n};
  return compute_impl(c, 1, off, box, periodic, pos, species, energy, forces, virial, stream);
}

int airebo_compute_static(airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species, const double* box,
                          const int32_t* periodic, double* energy, double* forces, double* virial, void* stream) {
  if (!c || (n > 0 && (!pos || !species || !forces)) || !energy || !virial || !box || !periodic)
    return fail(AIREBO_E_ARG, "null argument");
  if (n < 0) return fail(AIREBO_E_ARG, "n must be >= 0");
  return compute_static_impl(c, n, pos, species, box, periodic, energy, forces, virial, (hipStream_t)stream);
}

int airebo_compute_host(airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species, const double* box,
                        const int32_t* periodic, double* energy, double* forces, double* virial) {
  if (!c || (n > 0 && (!pos || !species || !forces)) || !energy || !virial || !box || !periodic)
    return fail(AIREBO_E_ARG, "null argument");
  if (n < 0 || n >= (1ll << 27)) return fail(AIREBO_E_ARG, "n out of range");
  HIPCHK(hipSetDevice(c->opt.device));
  size_t N = (size_t)std::max<int64_t>(n, 1);
  if (grow(c->hx, c->c_hx, 6 * N + 10) | grow(c->hs, c->c_hs, N)) return fail(AIREBO_E_DEVICE, "staging allocation");
  double* dpos = c->hx;
  double* dE = c->hx + 3 * N;
  double* dW = dE + 4;
  double* dF = dE + 10;
  if (n > 0) {
    HIPCHK(hipMemcpy(dpos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->hs, species, sizeof(int32_t) * n, hipMemcpyHostToDevice));
  }
  int rc = airebo_compute(c, n, dpos, c->hs, box, periodic, dE, dF, dW, nullptr);
  if (rc) return rc;
  HIPCHK(hipMemcpy(energy, dE, sizeof(double) * 4, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(virial, dW, sizeof(double) * 6, hipMemcpyDeviceToHost));
  if (n > 0) HIPCHK(hipMemcpy(forces, dF, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
  return 0;
}

int airebo_nve(airebo_ctx_t c, int64_t n, double* pos, double* vel, const int32_t* species, const double* box,
               const int32_t* periodic, const double* mass, double dt, int64_t nsteps, int64_t every,
               double* thermo, void* stream) {
  if (!c || (n > 0 && (!pos || !vel || !species)) || !mass || !box || !periodic)
    return fail(AIREBO_E_ARG, "null argument");
  if (n < 0 || nsteps < 0 || !(dt > 0) || !(mass[0] > 0) || !(mass[1] > 0))
    return fail(AIREBO_E_ARG, "bad n, step count, dt or mass");
  if (every > 0 && !thermo) return fail(AIREBO_E_ARG, "thermo output needed when thermo_every > 0");
  int64_t off[2] = {0, n};
  return nve_impl(c, 1, off, box, periodic, pos, vel, species, mass, dt, nsteps, every, thermo, stream);
}

int airebo_batch_compute(airebo_ctx_t c, int32_t nsys, const int64_t* sys_off, const double* boxes,
                         const int32_t* periodic, const double* pos, const int32_t* species, double* energy,
                         double* forces, double* virial, void* stream) {
  if (!c || nsys < 1 || !sys_off || !boxes || !periodic || !energy || !virial) return fail(AIREBO_E_ARG, "null argument");
  if (sys_off[nsys] > 0 && (!pos || !species || !forces)) return fail(AIREBO_E_ARG, "null argument");
  return compute_impl(c, nsys, sys_off, boxes, periodic, pos, species, energy, forces, virial, stream);
}

int airebo_batch_nve(airebo_ctx_t c, int32_t nsys, const int64_t* sys_off, const double* boxes,
                     const int32_t* periodic, double* pos, double* vel, const int32_t* species, const double* mass,
                     double dt, int64_t nsteps, int64_t every, double* thermo, void* stream) {
  if (!c || nsys < 1 || !sys_off || !boxes || !periodic || !mass) return fail(AIREBO_E_ARG, "null argument");
  if (sys_off[nsys] > 0 && (!pos || !vel || !species)) return fail(AIREBO_E_ARG, "null argument");
  if (nsteps < 0 || !(dt > 0) || !(mass[0] > 0) || !(mass[1] > 0)) return fail(AIREBO_E_ARG, "bad step count, dt or mass");
  if (every > 0 && !thermo) return fail(AIREBO_E_ARG, "thermo output needed when thermo_every > 0");
  return nve_impl(c, nsys, sys_off, boxes, periodic, pos, vel, species, mass, dt, nsteps, every, thermo, stream);
}

int airebo_md_begin(airebo_ctx_t c, int64_t n, const double* pos, const double* vel, const int32_t* species,
                    const double* box, const int32_t* periodic, const double* mass, double dt, void* stream) {
  if (!c || !pos || !vel || !species || !mass || !box || !periodic) return fail(AIREBO_E_ARG, "null argument");
  if (n < 1 || n >= (1ll << 27) || !(dt > 0) || !(mass[0] > 0) || !(mass[1] > 0))
    return fail(AIREBO_E_ARG, "bad n, dt or mass");
  int64_t off[2] = {0, n};
  return md_begin_airebo(c, 1, off, box, periodic, pos, vel, species, mass, dt, (hipStream_t)stream);
}

int airebo_batch_md_begin(airebo_ctx_t c, int32_t nsys, const int64_t* sys_off, const double* boxes,
                          const int32_t* periodic, const double* pos, const double* vel, const int32_t* species,
                          const double* mass, double dt, void* stream) {
  if (!c || nsys < 1 || !sys_off || !boxes || !periodic || !mass || !pos || !vel || !species)
    return fail(AIREBO_E_ARG, "null argument");
  if (sys_off[nsys] < 1 || !(dt > 0) || !(mass[0] > 0) || !(mass[1] > 0))
    return fail(AIREBO_E_ARG, "bad atom count, dt or mass");
  return md_begin_airebo(c, nsys, sys_off, boxes, periodic, pos, vel, species, mass, dt, (hipStream_t)stream);
}

int airebo_md_run(airebo_ctx_t c, int64_t nsteps, int64_t thermo_every, double* thermo, void* stream) {
  if (!c) return fail(AIREBO_E_ARG, "null argument");
  if (nsteps < 0 || thermo_every < 0) return fail(AIREBO_E_ARG, "bad step count");
  if (thermo_every > 0 && !thermo) return fail(AIREBO_E_ARG, "thermo output needed when thermo_every > 0");
  return md_run_impl(c, nsteps, thermo_every, thermo, (hipStream_t)stream);
}

int airebo_md_state(airebo_ctx_t c, double* pos, double* vel, void* stream) {
  if (!c) return fail(AIREBO_E_ARG, "null argument");
  return md_state_impl(c, pos, vel, (hipStream_t)stream);
}

void airebo_md_end(airebo_ctx_t c) {
  if (c) md_end_impl(c);
}

int airebo_profile_nve(airebo_ctx_t c, int64_t n, double* pos, double* vel, const int32_t* species,
                       const double* box, const int32_t* periodic, const double* mass, double dt, int64_t nsteps,
                       double* ms_out, int64_t* launches_out, void* stream) {
  if (!c || !ms_out || !launches_out) return fail(AIREBO_E_ARG, "null argument");
  c->prof = true;
  c->ev.clear();
  int rc = airebo_nve(c, n, pos, vel, species, box, periodic, mass, dt, nsteps, 0, nullptr, stream);
  c->prof = false;
  for (int k = 0; k < K_COUNT; ++k) { ms_out[k] = 0; launches_out[k] = 0; }
  for (auto& e : c->ev) {
    float ms = 0;
    if (rc == 0 && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ms_out[e.k] += ms;
      launches_out[e.k] += 1;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->ev.clear();
  return rc;
}

int airebo_kernel_count(void) { return K_COUNT; }

const char* airebo_kernel_name(int k) { return (k >= 0 && k < K_COUNT) ? kKernelNames[k] : ""; }

int airebo_stats(airebo_ctx_t c, int64_t* out) { return airebo_stats_n(c, out, 16); }

int airebo_stats_n(airebo_ctx_t c, int64_t* out, int n) {
  if (!c || !out) return fail(AIREBO_E_ARG, "null argument");
  if (n < 0) return fail(AIREBO_E_ARG, "negative count");
  for (int k = 0; k < n; ++k) out[k] = k < S_N ? (int64_t)c->host_stats[k] : 0;
  return std::min(n, (int)S_N);
}

}  // extern "C"

#include "surrogate.hip"
#include "peaks.hip"
