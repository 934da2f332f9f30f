// Learned surrogate of the AIREBO short-range energy (compiled as part of
// airebo.hip, after the AIREBO kernels and host code).
//
// E = sum_i E_NN(G_i; s_i) + E_far.  G_i: 112 symmetry functions of atom i:
//   radial   G[s*32 + m]      = sum_{j of species s, r < 6 A} exp(-eta (r - mu_m)^2) fc(r; 6)
//            mu_m = 0.8 + m (5.2/31) A, eta = 1 / (2 (2 * 5.2/31)^2)
//   angular  G[64 + t*16 + c] = 2^(1-zeta) sum_{j<k, s_j + s_k = t, r < 3.5 A}
//            (1 + lam cos theta_jik)^zeta exp(-eta_a (r_ij^2 + r_ik^2)) fc(r_ij; 3.5) fc(r_ik; 3.5)
//            c = 4 log2(zeta) + 2 [lam = -1] + [eta_a = 0.05], zeta in {1,2,4,8}, eta_a in {0.005, 0.05}
//   fc(r; R) = (1 + cos(pi r / R)) / 2.
// E_NN: per centre species, x = (G - mean) * istd, three SiLU layers of 64,
// linear output; E_i = scale * out + shift[s_i].  E_far: the LJ pair term
// (with its outer cutoff switch) times a cubic switch rising from 0 at 5 A to
// 1 at 6 A; no C_ij and no bond-order switch.
//
// An ensemble of networks gives the force spread; when its maximum over atoms
// exceeds the caller's threshold, the AIREBO kernels of the same context
// evaluate the step instead.  The decision is taken on the device, so a step
// stays one captured graph.
//
// Kernels: neighbour staging from the LJ list; descriptors and their
// Jacobian-vector product (lane per neighbour or neighbour pair, per-lane
// feature accumulators reduced by a butterfly reduce-scatter); descriptor
// vector-Jacobian product (forces; leg sums by shuffles, then one atomic per
// neighbour and component); the networks on BF16 MFMA 16x16x16 tiles with
// FP32 accumulation, both orientations of every weight matrix staged in LDS
// (inference: forward pass and input gradient; training: also the double
// backward of the force loss and the weight gradients); far-field pairs;
// ensemble mean and spread; Adam.

namespace airebo {
namespace nn {

constexpr int NRAD = 32, NANG = 16, DIM = 2 * NRAD + 3 * NANG;   // 112
constexpr int HID = 64;
constexpr int NM_MAX = 4;
constexpr float RAD_CUT = 6.0f, ANG_CUT = 3.5f;
constexpr double FAR0 = 5.0, FAR1 = 6.0;
constexpr int MAXNB = 192;      // neighbours within RAD_CUT kept per atom
constexpr int MAXANG = 48;      // neighbours within ANG_CUT
// parameter block of one species network (floats)
constexpr int OW1 = 0, OB1 = OW1 + HID * DIM, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + HID * HID, OW4 = OB3 + HID, OB4 = OW4 + HID, NPAR = OB4 + 1;
// accumulators of the surrogate (doubles, NSLOT copies)
enum { N_E = 0, N_EFAR = 4, N_VIR = 5, N_LOSSF = 11, N_A = 16 };
// padded LDS row strides (BF16 elements) against bank conflicts
constexpr int SD = DIM + 8, SH = HID + 8;   // LDS row strides: 16-byte rows for 8-element loads
constexpr float RAD_H = 5.2f / 31.0f;
constexpr float RAD_ETA = 1.0f / (2.0f * (2.0f * RAD_H) * (2.0f * RAD_H));

__device__ __forceinline__ float sig(float a) { return 1.0f / (1.0f + __expf(-a)); }
__device__ __forceinline__ float silu(float a) { return a * sig(a); }
// SiLU derivatives: d = s (1 + a (1 - s)), dd = s (1 - s) (2 + a (1 - 2 s))
__device__ __forceinline__ void silu_d(float a, float& d, float& dd) {
  float s = sig(a);
  d = s * (1.0f + a * (1.0f - s));
  dd = s * (1.0f - s) * (2.0f + a * (1.0f - 2.0f * s));
}
__device__ __forceinline__ unsigned short f2bf(float f) {   // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float fcut(float r, float rc, float& d) {
  if (r >= rc) { d = 0; return 0; }
  float s, c;
  sincospif(r / rc, &s, &c);
  d = -0.5f * (float)M_PI / rc * s;
  return 0.5f * (1.0f + c);
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sum over the 64 lanes of v[k] for every k; lane l returns the total of
// index l (butterfly reduce-scatter, 63 exchanges).  At stage S each lane
// keeps the half of its S-wide window selected by bit S of its lane index
// and adds the partner's copy of that half.
template <int S>
__device__ __forceinline__ void rs_stage(float (&v)[64], int lane) {
  bool up = lane & S;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    float send = up ? v[k] : v[k + S];
    float keep = up ? v[k + S] : v[k];
    v[k] = keep + __shfl_xor(send, S);
  }
  if constexpr (S > 1) rs_stage<S / 2>(v, lane);
}
__device__ __forceinline__ float reduce_scatter64(float (&v)[64]) {
  rs_stage<32>(v, threadIdx.x & (WAVE - 1));
  return v[0];
}

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct NbList {              // neighbours of one atom, staged in LDS by its wavefront
  int n, na;
  float dx[MAXNB], dy[MAXNB], dz[MAXNB], r[MAXNB];
  int j[MAXNB];
  signed char s[MAXNB];
  signed char aidx[MAXNB];   // index among the angular neighbours, or -1
  // angular neighbours (r < ANG_CUT): unit vector, length, cutoff value,
  // h_e = fc'(r)/r - 2 eta_e fc(r) and exp(-eta_e r^2) for eta_e = 0.005, 0.05
  float ux[MAXANG], uy[MAXANG], uz[MAXANG], ar[MAXANG], afc[MAXANG], ah0[MAXANG], ah1[MAXANG], ae0[MAXANG],
      ae1[MAXANG];
  int aj[MAXANG];            // atom of each angular neighbour
  signed char as[MAXANG];    // its species
};

// Far-field pair sums of one lane: energy (half per side), force on the
// centre, virial (half per side).
struct FarAcc {
  float e, f[3], W[6];
};

// Far-field pair term of one list entry beyond FAR0 and inside the LJ
// cutoff (FP32 arithmetic on the FP64 pair vector): half the energy and
// virial per side, the force on the centre.
__device__ __forceinline__ void far_pair(const DevParams& P, int p, double r2, float dx, float dy, float dz, float r,
                                         FarAcc& far) {
  if (!(r2 > FAR0 * FAR0 && r2 < P.rc2[p])) return;
  float V, dV, ds;
  lj_pair<float>(P, p, r, V, dV);
  float sw = 1.0f - Sw((r - (float)FAR0) * (float)(1.0 / (FAR1 - FAR0)), ds);
  ds = -ds * (float)(1.0 / (FAR1 - FAR0));
  float gr = (ds * V + sw * dV) * frcp(r);   // (dE_pair/dr) / r
  far.e += 0.5f * sw * V;
  far.f[0] += gr * dx; far.f[1] += gr * dy; far.f[2] += gr * dz;
  far.W[0] -= 0.5f * gr * dx * dx; far.W[1] -= 0.5f * gr * dy * dy; far.W[2] -= 0.5f * gr * dz * dz;
  far.W[3] -= 0.5f * gr * dx * dy; far.W[4] -= 0.5f * gr * dx * dz; far.W[5] -= 0.5f * gr * dy * dz;
}

// Stage the neighbours of atom i within RAD_CUT (image-resolved, from the LJ
// list's near part, in list order) in LDS, with the per-neighbour factors of
// the angular terms.  One wavefront.  With a far-field accumulator, the same
// pass adds the far-field pair term of every list entry beyond FAR0, and a
// second pass that of every entry of the list's far part.
__device__ void stage_nb(const Dev& D, int i, NbList& nb, const DevParams* P = nullptr, FarAcc* far = nullptr) {
  int lane = threadIdx.x & (WAVE - 1);
  unsigned long long below = lanes_below();
  double4 xi = D.x[i];
  int si = __double2int_rn(xi.w) == 0 ? 0 : 1;
  const SysBox& B = box_of(D, i);
  int nl = min(D.lj_n[i], D.lj_cap);
  int cnt = 0, cna = 0;
  // the next block of entries and positions is loaded while this one is used
  const unsigned* list = D.lj_e + (size_t)i * D.lj_cap;
  unsigned ent_n = lane < nl ? list[lane] : 0u;
  double4 xj_n = lane < nl ? D.x[ent_n & 0x7FFFFFFu] : xi;
  for (int base = 0; base < nl; base += WAVE) {
    int e = base + lane;
    bool ok = false, oka = false;
    float dx = 0, dy = 0, dz = 0, r = 0;
    int j = 0, sj = 0;
    unsigned ent = ent_n;
    double4 xj = xj_n;
    if (e + WAVE < nl) {
      ent_n = list[e + WAVE];
      xj_n = D.x[ent_n & 0x7FFFFFFu];
    }
    if (e < nl) {
      j = (int)(ent & 0x7FFFFFFu);
      int code = (int)(ent >> 27);
      double ddx = xj.x - xi.x + (code / 9 - 1) * B.L[0];
      double ddy = xj.y - xi.y + ((code / 3) % 3 - 1) * B.L[1];
      double ddz = xj.z - xi.z + (code % 3 - 1) * B.L[2];
      double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
      ok = r2 < (double)RAD_CUT * RAD_CUT;
      oka = r2 < (double)ANG_CUT * ANG_CUT;
      dx = (float)ddx; dy = (float)ddy; dz = (float)ddz; r = (float)sqrt(r2);
      sj = __double2int_rn(xj.w) == 0 ? 0 : 1;   // invalid codes are reported by k_load
      if (far) far_pair(*P, si + sj, r2, dx, dy, dz, r, *far);
    }
    unsigned long long m = __ballot(ok);
    unsigned long long ma = __ballot(oka);
    int pos = cnt + __popcll(m & below);
    int posa = cna + __popcll(ma & below);
    if (ok && pos < MAXNB) {
      nb.dx[pos] = dx; nb.dy[pos] = dy; nb.dz[pos] = dz; nb.r[pos] = r; nb.j[pos] = j;
      nb.s[pos] = (signed char)sj;
      bool a = oka && posa < MAXANG;
      nb.aidx[pos] = a ? (signed char)posa : (signed char)-1;
      if (a) {
        float ir = frcp(r), dfc;
        float fc = fcut(r, ANG_CUT, dfc);
        nb.ux[posa] = dx * ir; nb.uy[posa] = dy * ir; nb.uz[posa] = dz * ir;
        nb.ar[posa] = r;
        nb.afc[posa] = fc;
        nb.ah0[posa] = dfc * ir - 2.0f * 0.005f * fc;
        nb.ah1[posa] = dfc * ir - 2.0f * 0.05f * fc;
        nb.ae0[posa] = __expf(-0.005f * r * r);
        nb.ae1[posa] = __expf(-0.05f * r * r);
        nb.aj[posa] = j;
        nb.as[posa] = (signed char)sj;
      }
    }
    cnt += __popcll(m);
    cna += __popcll(ma);
  }
  // the far part of the LJ list (beyond 3 max R2 > RAD_CUT): far field only
  if (far) {
    const int nf = min(D.lf_n[i], D.lf_cap);
    const unsigned* lf = D.lf_e + (size_t)i * D.lf_cap;
    for (int e = lane; e < nf; e += WAVE) {
      unsigned ent = lf[e];
      double4 xj = D.x[ent & 0x7FFFFFFu];
      int code = (int)(ent >> 27);
      double ddx = xj.x - xi.x + (code / 9 - 1) * B.L[0];
      double ddy = xj.y - xi.y + ((code / 3) % 3 - 1) * B.L[1];
      double ddz = xj.z - xi.z + (code % 3 - 1) * B.L[2];
      double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
      int sj = __double2int_rn(xj.w) == 0 ? 0 : 1;
      far_pair(*P, si + sj, r2, (float)ddx, (float)ddy, (float)ddz, (float)sqrt(r2), *far);
    }
  }
  if (lane == 0) {
    if (cnt > MAXNB || cna > MAXANG) atomicOr(D.flags, F_OV_NN);
    nb.n = min(cnt, MAXNB);
    nb.na = min(cna, MAXANG);
  }
  wave_sync();
}

// Pair index p of the upper triangle (a < b < na) -> (a, b).
__device__ __forceinline__ void tri_decode(int p, int na, int& a, int& b) {
  float m = 2.0f * na - 1.0f;
  int r = (int)((m - sqrtf(fmaxf(m * m - 8.0f * p, 0.0f))) * 0.5f);
  r = max(0, min(r, na - 2));
  auto start = [&](int q) { return q * na - q * (q + 1) / 2; };
  while (r > 0 && start(r) > p) --r;
  while (r < na - 2 && start(r + 1) <= p) ++r;
  a = r;
  b = p - start(r) + r + 1;
}

// (1 + lam c)^zeta and its derivative in c for zeta = 1, 2, 4, 8.
__device__ __forceinline__ void ang_pows(float base, float lam, float (&P)[4], float (&dP)[4]) {
  float b2 = base * base, b4 = b2 * b2;
  P[0] = base; P[1] = b2; P[2] = b4; P[3] = b4 * b4;
  dP[0] = lam; dP[1] = 2.0f * lam * base; dP[2] = 4.0f * lam * b2 * base; dP[3] = 8.0f * lam * b4 * b2 * base;
}
__device__ __forceinline__ float ang_pre(int zi) { return zi == 0 ? 1.0f : (zi == 1 ? 0.5f : (zi == 2 ? 0.125f : 0.0078125f)); }

// Angular factors of the neighbour pair (a, b): cos theta, the products
// pe_c = 2^(1-zeta) exp(-eta_e (r_a^2 + r_b^2)) times (1 + lam cos)^zeta (w2)
// and times its cos-derivative (w1), feature c = 4 zi + 2 li + ei.
struct PairAng {
  float cs, w1[NANG], w2[NANG];
};
__device__ __forceinline__ void pair_ang(const NbList& nb, int a, int b, PairAng& Q) {
  Q.cs = nb.ux[a] * nb.ux[b] + nb.uy[a] * nb.uy[b] + nb.uz[a] * nb.uz[b];
  float E[2] = {nb.ae0[a] * nb.ae0[b], nb.ae1[a] * nb.ae1[b]};
  float P[2][4], dP[2][4];
  ang_pows(1.0f + Q.cs, 1.0f, P[0], dP[0]);
  ang_pows(1.0f - Q.cs, -1.0f, P[1], dP[1]);
#pragma unroll
  for (int zi = 0; zi < 4; ++zi)
#pragma unroll
    for (int li = 0; li < 2; ++li)
#pragma unroll
      for (int ei = 0; ei < 2; ++ei) {
        int c = 4 * zi + 2 * li + ei;
        float pe = ang_pre(zi) * E[ei];
        Q.w1[c] = pe * dP[li][zi];
        Q.w2[c] = pe * P[li][zi];
      }
}

// Descriptors (MODE 0) or their Jacobian-vector product with w [n][3]
// (MODE 1): out[i][f] = sum_a dG_if/dx_a . w_a.  One wavefront per atom.
// The descriptors take a register budget for six wavefronts per SIMD (what
// the LDS of four-atom blocks allows; a small spill).
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 6 : 1, 8)))
void k_desc(Dev D, float* __restrict__ out, const float* __restrict__ w) {
  __shared__ NbList nbs[4];
  int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
  int i = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  if (i >= D.n) return;
  NbList& nb = nbs[wv];
  stage_nb(D, i, nb);
  float wi0 = 0, wi1 = 0, wi2 = 0;
  if (MODE == 1) { wi0 = w[3 * i]; wi1 = w[3 * i + 1]; wi2 = w[3 * i + 2]; }
  float v[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) v[k] = 0.0f;
  // radial: lane per neighbour
  for (int q = lane; q < nb.n; q += WAVE) {
    float r = nb.r[q], dfc;
    float fcv = fcut(r, RAD_CUT, dfc);
    float w0 = nb.s[q] == 0 ? 1.0f : 0.0f, w1 = 1.0f - w0;
    float proj = 0.0f;
    if (MODE == 1) {
      int j = nb.j[q];
      proj = (nb.dx[q] * (w[3 * j] - wi0) + nb.dy[q] * (w[3 * j + 1] - wi1) + nb.dz[q] * (w[3 * j + 2] - wi2)) *
             frcp(r);
    }
#pragma unroll
    for (int m = 0; m < NRAD; ++m) {
      float t = r - (0.8f + m * RAD_H);
      float g = __expf(-RAD_ETA * t * t);
      float val = MODE == 0 ? g * fcv : g * (fcv * (-2.0f * RAD_ETA * t) + dfc) * proj;
      v[m] += w0 * val;
      v[NRAD + m] += w1 * val;
    }
  }
  float tot = reduce_scatter64(v);
  out[(size_t)i * DIM + lane] = tot;
  // angular: lane per neighbour pair
#pragma unroll
  for (int k = 0; k < 64; ++k) v[k] = 0.0f;
  int na = nb.na, npair = na * (na - 1) / 2;
  for (int p = lane; p < npair; p += WAVE) {
    int a, b;
    tri_decode(p, na, a, b);
    int t = nb.as[a] + nb.as[b];
    float t0 = t == 0 ? 1.0f : 0.0f, t1 = t == 1 ? 1.0f : 0.0f, t2 = t == 2 ? 1.0f : 0.0f;
    PairAng Q;
    pair_ang(nb, a, b, Q);
    float ff = nb.afc[a] * nb.afc[b];
    float A = 0, Ba = 0, Bb = 0;   // JVP pieces
    if (MODE == 1) {
      int ja = nb.aj[a], jb = nb.aj[b];
      float ajx = w[3 * ja] - wi0, ajy = w[3 * ja + 1] - wi1, ajz = w[3 * ja + 2] - wi2;
      float akx = w[3 * jb] - wi0, aky = w[3 * jb + 1] - wi1, akz = w[3 * jb + 2] - wi2;
      float ua_j = nb.ux[a] * ajx + nb.uy[a] * ajy + nb.uz[a] * ajz;   // u_a . a_j / r_a
      float ub_j = nb.ux[b] * ajx + nb.uy[b] * ajy + nb.uz[b] * ajz;
      float ua_k = nb.ux[a] * akx + nb.uy[a] * aky + nb.uz[a] * akz;
      float ub_k = nb.ux[b] * akx + nb.uy[b] * aky + nb.uz[b] * akz;   // u_b . a_k / r_b
      A = ff * ((ub_j - Q.cs * ua_j) * frcp(nb.ar[a]) + (ua_k - Q.cs * ub_k) * frcp(nb.ar[b]));
      Ba = nb.afc[b] * nb.ar[a] * ua_j;
      Bb = nb.afc[a] * nb.ar[b] * ub_k;
    }
#pragma unroll
    for (int c = 0; c < NANG; ++c) {
      float val;
      if (MODE == 0) {
        val = Q.w2[c] * ff;
      } else {
        int ei = c & 1;
        float ha = ei ? nb.ah1[a] : nb.ah0[a], hb = ei ? nb.ah1[b] : nb.ah0[b];
        val = Q.w1[c] * A + Q.w2[c] * (ha * Ba + hb * Bb);
      }
      v[c] += t0 * val;
      v[16 + c] += t1 * val;
      v[32 + c] += t2 * val;
    }
  }
  tot = reduce_scatter64(v);
  if (lane < 3 * NANG) out[(size_t)i * DIM + 2 * NRAD + lane] = tot;
}

// Descriptor vector-Jacobian product: F[m][a] = -sum_{i,f} g[m][i][f] dG_if/dx_a
// for nm sets g ([nm][n][DIM], complete before the launch); F ([nm][n][3],
// FP32) must start at zero.  The
// virial of the mean over the sets (sum over contributions of
// (x_a - x_i) (x) F_a) goes to acc[slot][N_VIR..].  One wavefront per centre
// atom i.
//   angular: lane per neighbour pair (a, b) forms dE/du_a and dE/du_b; the
//     legs' sums are formed by shuffles (a segmented scan along each row of
//     the pair triangle, a gather down its columns) and each leg's force is
//     added to its atom (one atomic per component and set);
//   radial: gathered from both ends of each pair (the neighbour's dE/dG
//     slice is read from memory), no atomics.
// The centre's own force is a wavefront sum.
// With FAR, the same pass over the LJ list evaluates the far-field term into
// Ff [n][3] and acc.
// One wavefront per block, register budget for four wavefronts per SIMD
// (a few registers spill; three per SIMD without the bound, and a budget for
// five spills heavily).  The centre's dE/dG rows are staged in LDS: the
// angular and radial terms index them by the species of the pair or the
// neighbour, which differs between lanes (a per-lane select of global
// addresses made every pair wait on its own loads: ~2/3 of the kernel).
template <bool FAR>
__global__ __launch_bounds__(WAVE, 4) void k_desc_force(Dev D, const DevParams* __restrict__ Pp, const float* __restrict__ g,
                                                     int nm, float* __restrict__ F, double* __restrict__ Ff,
                                                     double* __restrict__ acc) {
  __shared__ NbList nb;
  __shared__ float gc[NM_MAX][DIM];        // the centre's dE/dG rows (read with per-lane indices)
  int lane = threadIdx.x;
  const int i = blockIdx.x;
  if (i >= D.n) return;
  float W[6] = {0, 0, 0, 0, 0, 0};
  FarAcc far = {0, {0, 0, 0}, {0, 0, 0, 0, 0, 0}};
  const size_t mstride = (size_t)D.n * DIM;
  const float* gi = g + (size_t)i * DIM;   // row of model m: gi + m * mstride
  for (int k = lane; k < nm * DIM; k += WAVE) gc[k / DIM][k % DIM] = gi[(k / DIM) * mstride + k % DIM];
  stage_nb(D, i, nb, Pp, FAR ? &far : nullptr);   // ends with a wavefront barrier
  const float inm = 1.0f / nm;
  float fi[NM_MAX][3] = {};
  float lf[NM_MAX][3] = {};   // force on leg `lane` (lane < na)
  int na = nb.na, npair = na * (na - 1) / 2;
  auto start = [&](int q) { return q * na - q * (q + 1) / 2; };
  // ---- angular: lane per pair (a, b), a < b, in blocks of 64 pairs.  The
  // pairs of one row a are consecutive lanes: a segmented scan leaves the
  // row's sum of -dE/du_a in its last lane, which leg lane a reads; each row
  // of the block holds at most one pair (r, b) for a given b, read by leg
  // lane b.  All in registers (shuffles), one set at a time.
  for (int base = 0; base < npair; base += WAVE) {
    int p = base + lane;
    bool live = p < npair;
    int a = 0, b = 1;
    if (live) tri_decode(p, na, a, b);
    PairAng Q;
    pair_ang(nb, a, b, Q);   // in range for every lane (a < b < na), used only when live
    int t = nb.as[a] + nb.as[b];
    float fa = nb.afc[a], fb = nb.afc[b], ra = nb.ar[a], rb = nb.ar[b];
    float ira = frcp(ra), irb = frcp(rb);
    float uax = nb.ux[a], uay = nb.uy[a], uaz = nb.uz[a], ubx = nb.ux[b], uby = nb.uy[b], ubz = nb.uz[b];
    float ha0 = nb.ah0[a], ha1 = nb.ah1[a], hb0 = nb.ah0[b], hb1 = nb.ah1[b];
    // block-uniform layout: first lane of this lane's row segment; for leg
    // lane `lane`, the last lane of its row in the block; the rows present
    int seg0 = live ? max(start(a), base) - base : lane;
    int rs = start(lane);
    int rlo = max(rs, base), rhi = min(rs + na - 1 - lane, min(base + WAVE, npair));
    bool has_row = lane < na - 1 && rhi > rlo;
    int row_src = has_row ? rhi - 1 - base : lane;
    int r_first, r_last, dummy;
    tri_decode(base, na, r_first, dummy);
    tri_decode(min(base + WAVE, npair) - 1, na, r_last, dummy);
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m)
      if (m < nm) {
        float gux = 0, guy = 0, guz = 0, gvx = 0, gvy = 0, gvz = 0;
        if (live) {
          const float* ga = &gc[m][2 * NRAD + t * NANG];   // LDS, indexed by the pair's species sum
          float S1 = 0, S20 = 0, S21 = 0;
#pragma unroll
          for (int c = 0; c < NANG; ++c) {
            float gv = ga[c];
            S1 += gv * Q.w1[c];
            if (c & 1) S21 += gv * Q.w2[c]; else S20 += gv * Q.w2[c];
          }
          float Ac = fa * fb * S1;
          float Ba = fb * (ha0 * S20 + ha1 * S21) * ra;
          float Bb = fa * (hb0 * S20 + hb1 * S21) * rb;
          // dE/du_a and dE/du_b (u = vector from the centre to the neighbour)
          float ca = Ac * ira, cb = Ac * irb;
          gux = ca * (ubx - Q.cs * uax) + Ba * uax;
          guy = ca * (uby - Q.cs * uay) + Ba * uay;
          guz = ca * (ubz - Q.cs * uaz) + Ba * uaz;
          gvx = cb * (uax - Q.cs * ubx) + Bb * ubx;
          gvy = cb * (uay - Q.cs * uby) + Bb * uby;
          gvz = cb * (uaz - Q.cs * ubz) + Bb * ubz;
          fi[m][0] += gux + gvx; fi[m][1] += guy + gvy; fi[m][2] += guz + gvz;
          W[0] -= inm * (ra * uax * gux + rb * ubx * gvx);
          W[1] -= inm * (ra * uay * guy + rb * uby * gvy);
          W[2] -= inm * (ra * uaz * guz + rb * ubz * gvz);
          W[3] -= inm * (ra * uax * guy + rb * ubx * gvy);
          W[4] -= inm * (ra * uax * guz + rb * ubx * gvz);
          W[5] -= inm * (ra * uay * guz + rb * uby * gvz);
        }
        // row sums of -dE/du_a: segmented inclusive scan
        float sx = -gux, sy = -guy, sz = -guz;
        for (int o = 1; o < WAVE; o <<= 1) {
          float tx = __shfl_up(sx, o), ty = __shfl_up(sy, o), tz = __shfl_up(sz, o);
          if (lane - o >= seg0) { sx += tx; sy += ty; sz += tz; }
        }
        {
          float tx = __shfl(sx, row_src), ty = __shfl(sy, row_src), tz = __shfl(sz, row_src);
          if (has_row) { lf[m][0] += tx; lf[m][1] += ty; lf[m][2] += tz; }
        }
        // column terms -dE/du_b: pair (r, lane) of each row r in the block
        for (int r = r_first; r <= r_last; ++r) {
          int q = start(r) + lane - r - 1;
          bool ok = lane < na && lane > r && q >= base && q < base + WAVE && q < npair;
          int src = ok ? q - base : lane;
          float tx = __shfl(-gvx, src), ty = __shfl(-gvy, src), tz = __shfl(-gvz, src);
          if (ok) { lf[m][0] += tx; lf[m][1] += ty; lf[m][2] += tz; }
        }
      }
  }
  // angular legs: force on each leg atom, one atomic per component and set
  if (lane < na) {
    int ja = nb.aj[lane];
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m)
      if (m < nm) {
        float* Fj = F + ((size_t)m * D.n + ja) * 3;
        atomicAdd(Fj, lf[m][0]); atomicAdd(Fj + 1, lf[m][1]); atomicAdd(Fj + 2, lf[m][2]);
      }
  }
  // ---- radial, gathered: lane per neighbour j.  Both E_i (through G_i[s_j])
  // and E_j (through G_j[s_i]) depend on r_ij; every pair is visited from
  // both ends, and each end applies the full pair force to its own atom and
  // half of the pair virial.
  const int si = __double2int_rn(D.x[i].w) == 0 ? 0 : 1;
  for (int q = lane; q < nb.n; q += WAVE) {
    float r = nb.r[q], dfc;
    float fcv = fcut(r, RAD_CUT, dfc);
    int sp = nb.s[q], j = nb.j[q];
    float dg[NRAD];
#pragma unroll
    for (int k = 0; k < NRAD; ++k) {
      float t = r - (0.8f + k * RAD_H);
      dg[k] = __expf(-RAD_ETA * t * t) * (fcv * (-2.0f * RAD_ETA * t) + dfc);
    }
    float ir = frcp(r);
    float ux = nb.dx[q] * ir, uy = nb.dy[q] * ir, uz = nb.dz[q] * ir;
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m)
      if (m < nm) {
        const float* gm = &gc[m][sp * NRAD];                                    // centre, LDS
        const float* gj = g + m * mstride + (size_t)j * DIM + si * NRAD;       // neighbour, vector loads
        float de = 0;
#pragma unroll
        for (int k4 = 0; k4 < NRAD / 4; ++k4) {
          float4 v = *reinterpret_cast<const float4*>(gj + 4 * k4);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            int kk = 4 * k4 + k;
            float own = gm[kk];
            float oth = k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
            de += (own + oth) * dg[kk];
          }
        }
        // dE/dr_ij > 0 pulls i towards j: F_i = +dE/dr u
        fi[m][0] += de * ux; fi[m][1] += de * uy; fi[m][2] += de * uz;
        float h = -0.5f * inm * de;   // half pair virial: d (x) F_j with F_j = -dE/dr u
        W[0] += h * nb.dx[q] * ux; W[1] += h * nb.dy[q] * uy; W[2] += h * nb.dz[q] * uz;
        W[3] += h * nb.dx[q] * uy; W[4] += h * nb.dx[q] * uz; W[5] += h * nb.dy[q] * uz;
      }
  }
#pragma unroll
  for (int m = 0; m < NM_MAX; ++m)
    if (m < nm)
      for (int c = 0; c < 3; ++c) {
        float s = fi[m][c];
        for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) atomicAdd(&F[((size_t)m * D.n + i) * 3 + c], s);
      }
  int slot = (blockIdx.x & (NSLOT - 1)) * N_A;
  if (FAR) {
    for (int c = 0; c < 3; ++c) {
      double s = far.f[c];
      for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) Ff[3 * i + c] = s;
    }
    double s = far.e;
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && s != 0) atomic_add(&acc[slot + N_EFAR], s);
  }
  for (int c = 0; c < 6; ++c) {
    double s = (double)W[c] + (double)far.W[c];
    for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0 && s != 0) atomic_add(&acc[slot + N_VIR + c], s);
  }
}

// ---------------------------------------------------------------------------
// Network tiles on the BF16 matrix cores: MFMA 16x16x32 (gfx950) for every
// full 32-deep slice of K, 16x16x16 for a 16-deep remainder.  16x16x32: lane
// l holds A[l % 16][8 (l / 16) + v] and B[8 (l / 16) + v][l % 16], v = 0..7;
// 16x16x16: A[l % 16][4 (l / 16) + v] and B[4 (l / 16) + v][l % 16],
// v = 0..3; both give D[4 (l / 16) + v][l % 16], v = 0..3.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// D = A B for one 16x16 tile (A, B row-major FP32, rounded to BF16): a check
// of the lane layout above.  One wavefront.
__global__ void k_mfma_check(const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ Dout) {
  int l = threadIdx.x;
  bf16x4 a, b;
  for (int v = 0; v < 4; ++v) {
    a[v] = (short)f2bf(A[(l % 16) * 16 + 4 * (l / 16) + v]);
    b[v] = (short)f2bf(B[(4 * (l / 16) + v) * 16 + l % 16]);
  }
  f32x4 d = {0, 0, 0, 0};
  d = mfma(a, b, d);
  for (int v = 0; v < 4; ++v) Dout[(4 * (l / 16) + v) * 16 + l % 16] = d[v];
}

// The same for the 16x16x32 tile: A [16][32], B [32][16] row-major FP32.
__global__ void k_mfma32_check(const float* __restrict__ A, const float* __restrict__ B, float* __restrict__ Dout) {
  int l = threadIdx.x;
  bf16x8 a, b;
  for (int v = 0; v < 8; ++v) {
    a[v] = __builtin_bit_cast(__bf16, f2bf(A[(l % 16) * 32 + 8 * (l / 16) + v]));
    b[v] = __builtin_bit_cast(__bf16, f2bf(B[(8 * (l / 16) + v) * 16 + l % 16]));
  }
  f32x4 d = {0, 0, 0, 0};
  d = mfma32(a, b, d);
  for (int v = 0; v < 4; ++v) Dout[(4 * (l / 16) + v) * 16 + l % 16] = d[v];
}

// Weights of one species network in LDS: BF16, both orientations (rows padded).
struct __attribute__((aligned(16))) NetLDS {
  unsigned short W1[HID * SD], W1T[DIM * SH], W2[HID * SH], W2T[HID * SH], W3[HID * SH], W3T[HID * SH];
  float b1[HID], b2[HID], b3[HID], w4[HID], b4;
};
struct __attribute__((aligned(16))) TileLDS {   // per-wave staging of one tile
  unsigned short X[16 * SD];
  unsigned short H[16 * SH];
  int rows[16];
};

__device__ void load_net(NetLDS& N, const float* __restrict__ P, int t, int nt) {
  for (int k = t; k < HID * DIM; k += nt) {
    int o = k / DIM, f = k % DIM;
    unsigned short v = f2bf(P[OW1 + k]);
    N.W1[o * SD + f] = v;
    N.W1T[f * SH + o] = v;
  }
  for (int k = t; k < HID * HID; k += nt) {
    int o = k / HID, f = k % HID;
    unsigned short v2 = f2bf(P[OW2 + k]), v3 = f2bf(P[OW3 + k]);
    N.W2[o * SH + f] = v2; N.W2T[f * SH + o] = v2;
    N.W3[o * SH + f] = v3; N.W3T[f * SH + o] = v3;
  }
  for (int k = t; k < HID; k += nt) {
    N.b1[k] = P[OB1 + k]; N.b2[k] = P[OB2 + k]; N.b3[k] = P[OB3 + k]; N.w4[k] = P[OW4 + k];
  }
  if (t == 0) N.b4 = P[OB4];
}

// Y[16 x NO] = X[16 x K] W^T, W [NO][K] (row stride SW), X [16][K] (row
// stride SX), both BF16 in LDS.  y[ct][v] = Y[4 (l / 16) + v][16 ct + l % 16].
template <int K, int NO, int SX, int SW>
__device__ __forceinline__ void mm(const unsigned short* X, const unsigned short* W, f32x4 (&y)[NO / 16]) {
  static_assert(K % 16 == 0 && (SX * 2) % 16 == 0 && (SW * 2) % 16 == 0, "tile shapes and 16-byte rows");
  int l = threadIdx.x & (WAVE - 1);
  int row = l % 16, g = l / 16;
#pragma unroll
  for (int ct = 0; ct < NO / 16; ++ct) y[ct] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int kt = 0; kt < K / 32; ++kt) {
    bf16x8 a = *reinterpret_cast<const bf16x8*>(X + row * SX + kt * 32 + 8 * g);
#pragma unroll
    for (int ct = 0; ct < NO / 16; ++ct) {
      bf16x8 b = *reinterpret_cast<const bf16x8*>(W + (ct * 16 + row) * SW + kt * 32 + 8 * g);
      y[ct] = mfma32(a, b, y[ct]);
    }
  }
  if constexpr (K % 32 == 16) {   // the last 16 of K
    constexpr int k0 = K - 16;
    bf16x4 a = *reinterpret_cast<const bf16x4*>(X + row * SX + k0 + 4 * g);
#pragma unroll
    for (int ct = 0; ct < NO / 16; ++ct) {
      bf16x4 b = *reinterpret_cast<const bf16x4*>(W + (ct * 16 + row) * SW + k0 + 4 * g);
      y[ct] = mfma(a, b, y[ct]);
    }
  }
}

// Store D-layout tiles as BF16 rows [16][NO] (row stride S).
template <int NO, int S>
__device__ __forceinline__ void put(unsigned short* X, const f32x4 (&y)[NO / 16]) {
  int l = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int ct = 0; ct < NO / 16; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(4 * (l / 16) + v) * S + ct * 16 + l % 16] = f2bf(y[ct][v]);
}

struct NNArgs {
  int n;
  const int* order;            // [2][n]: atoms of species 0, then of species 1
  const int* cnt;              // [2] atoms per species
  const float* G;              // [n][DIM]
  const float* mean;           // [DIM]
  const float* istd;           // [DIM]
  const float* params;         // [nm][2][NPAR]
  float scale;
  const float* shift;          // [2]
  float* E;                    // [nm][n] per-atom energies
  float* dEdG;                 // [nm][n][DIM]
  // training
  const float* U;              // [nm][n][DIM]: descriptor JVP of the force-loss adjoint
  const float* dE;             // [nm]: energy-loss adjoint
  float* grad;                 // [nm][2][NPAR]
};

// Pre-activations a1..a3, input-side gradients ga1..ga3 (gradient of the
// output with respect to a_k) and gh1, gh2 (with respect to h_1, h_2) of one
// tile, D layout.
struct TileState {
  f32x4 a1[4], a2[4], a3[4], ga1[4], ga2[4], ga3[4], gh1[4], gh2[4];
};

__device__ __forceinline__ void tile_rows(const NNArgs& A, int sp, int tile, TileLDS& T) {
  int l = threadIdx.x & (WAVE - 1);
  if (l < 16) {
    int k = tile * 16 + l;
    T.rows[l] = k < A.cnt[sp] ? A.order[(size_t)sp * A.n + k] : -1;
  }
  wave_sync();
}

// Forward pass and input gradient of one tile of 16 atoms, one wavefront.
__device__ __forceinline__ void tile_fwd_bwd(const NNArgs& A, const NetLDS& N, TileLDS& T, int model, int sp,
                                             TileState& S) {
  int l = threadIdx.x & (WAVE - 1);
  int c0 = l % 16, rg = 4 * (l / 16);
  for (int k = l; k < 16 * DIM; k += WAVE) {
    int r = k / DIM, f = k % DIM;
    int at = T.rows[r];
    float v = at >= 0 ? (A.G[(size_t)at * DIM + f] - A.mean[f]) * A.istd[f] : 0.0f;
    T.X[r * SD + f] = f2bf(v);
  }
  wave_sync();
  f32x4 h[4];
  mm<DIM, HID, SD, SD>(T.X, N.W1, S.a1);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) { S.a1[ct][v] += N.b1[ct * 16 + c0]; h[ct][v] = silu(S.a1[ct][v]); }
  wave_sync();
  put<HID, SH>(T.H, h);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W2, S.a2);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) { S.a2[ct][v] += N.b2[ct * 16 + c0]; h[ct][v] = silu(S.a2[ct][v]); }
  wave_sync();
  put<HID, SH>(T.H, h);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W3, S.a3);
  float erow[4] = {0, 0, 0, 0};
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      S.a3[ct][v] += N.b3[ct * 16 + c0];
      float d, dd;
      silu_d(S.a3[ct][v], d, dd);
      erow[v] += N.w4[ct * 16 + c0] * silu(S.a3[ct][v]);
      S.ga3[ct][v] = N.w4[ct * 16 + c0] * d;
    }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    for (int o = 8; o > 0; o >>= 1) erow[v] += __shfl_xor(erow[v], o);   // over the 16 columns of the group
  if (c0 == 0)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int at = T.rows[rg + v];
      if (at >= 0) A.E[(size_t)model * A.n + at] = A.scale * (erow[v] + N.b4) + A.shift[sp];
    }
  // input gradient: gh2 = ga3 W3, ga2 = gh2 s'(a2), gh1 = ga2 W2, ga1 = gh1 s'(a1), gG = ga1 W1
  wave_sync();
  put<HID, SH>(T.H, S.ga3);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W3T, S.gh2);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a2[ct][v], d, dd);
      S.ga2[ct][v] = S.gh2[ct][v] * d;
    }
  wave_sync();
  put<HID, SH>(T.H, S.ga2);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W2T, S.gh1);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a1[ct][v], d, dd);
      S.ga1[ct][v] = S.gh1[ct][v] * d;
    }
  wave_sync();
  put<HID, SH>(T.H, S.ga1);
  wave_sync();
  f32x4 gG[DIM / 16];
  mm<HID, DIM, SH, SH>(T.H, N.W1T, gG);
#pragma unroll
  for (int ct = 0; ct < DIM / 16; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int at = T.rows[rg + v];
      int f = ct * 16 + c0;
      if (at >= 0) A.dEdG[((size_t)model * A.n + at) * DIM + f] = gG[ct][v] * A.scale * A.istd[f];
    }
  wave_sync();
}

// BF16 images of every (model, species) network in the LDS layout, built
// once per weight update; inference blocks copy their image linearly.
__global__ void k_pack(const float* __restrict__ params, NetLDS* __restrict__ out) {
  load_net(out[blockIdx.x], params + (size_t)blockIdx.x * NPAR, threadIdx.x, blockDim.x);
}

// Inference: grid (blocks, 2 nm), blockIdx.y = 2 model + species; each block
// copies that network's image into LDS once and its waves walk the species'
// tiles.
constexpr int MLP_WAVES = 8;
__global__ __launch_bounds__(64 * MLP_WAVES) void k_mlp(NNArgs A, const NetLDS* __restrict__ packed) {
  __shared__ NetLDS N;
  __shared__ TileLDS Ts[MLP_WAVES];
  int model = blockIdx.y >> 1, sp = blockIdx.y & 1;
  int ntile = (A.cnt[sp] + 15) / 16;
  if ((int)blockIdx.x * MLP_WAVES >= ntile) return;   // whole block
  {
    const uint4* src = reinterpret_cast<const uint4*>(packed + blockIdx.y);
    uint4* dst = reinterpret_cast<uint4*>(&N);
    for (int k = threadIdx.x; k < (int)(sizeof(NetLDS) / 16); k += blockDim.x) dst[k] = src[k];
  }
  __syncthreads();
  int wv = threadIdx.x / WAVE;
  for (int tile = blockIdx.x * MLP_WAVES + wv; tile < ntile; tile += gridDim.x * MLP_WAVES) {
    tile_rows(A, sp, tile, Ts[wv]);
    TileState S;
    tile_fwd_bwd(A, N, Ts[wv], model, sp, S);
  }
}

// Training: one wavefront per tile (blockIdx.x over the tiles of both
// species, blockIdx.y = model).  Besides the forward pass and input gradient
// it forms the gradient, with respect to every weight, of
// sum_i u_i . dE_i/dG_i (the force-loss term; u = descriptor JVP of the force
// adjoint) plus the energy loss:
//   tangent along un = u scale istd:  q1 = W1 un, p1 = s'(a1) q1, q2 = W2 p1,
//     p2 = s'(a2) q2, q3 = W3 p2;
//   second-order terms  r_k = q_k gh_k s''(a_k)  (gh3 = w4);
//   adjoints  A3 = dE ga3 + r3,  A2 = (A3 W3) s'(a2) + r2,  A1 = (A2 W2) s'(a1) + r1;
//   dW1 = A1^T x + ga1^T un,  dW2 = A2^T h1 + ga2^T p1,  dW3 = A3^T h2 + ga3^T p2,
//   dw4 = dE h3 + s'(a3) q3,  db_k = sum_rows A_k,  db4 = sum_rows dE
//   (dE is the energy adjoint times scale).
__global__ __launch_bounds__(64) void k_mlp_train(NNArgs A) {
  __shared__ NetLDS N;
  __shared__ TileLDS T;
  __shared__ float RA[16][HID], RB[16][HID], RC[16][HID];
  __shared__ float XN[16][DIM], UN[16][DIM];
  int model = blockIdx.y;
  int nt0 = (A.cnt[0] + 15) / 16, nt1 = (A.cnt[1] + 15) / 16;
  int sp = (int)blockIdx.x < nt0 ? 0 : 1;
  int tile = sp ? (int)blockIdx.x - nt0 : (int)blockIdx.x;
  if (sp == 1 && tile >= nt1) return;
  int l = threadIdx.x;
  int c0 = l % 16, rg = 4 * (l / 16);
  load_net(N, A.params + ((size_t)model * 2 + sp) * NPAR, l, WAVE);
  wave_sync();
  tile_rows(A, sp, tile, T);
  TileState S;
  tile_fwd_bwd(A, N, T, model, sp, S);
  const float sc = A.scale;
  for (int k = l; k < 16 * DIM; k += WAVE) {
    int r = k / DIM, f = k % DIM;
    int at = T.rows[r];
    XN[r][f] = at >= 0 ? (A.G[(size_t)at * DIM + f] - A.mean[f]) * A.istd[f] : 0.0f;
    float u = at >= 0 ? A.U[((size_t)model * A.n + at) * DIM + f] * sc * A.istd[f] : 0.0f;
    UN[r][f] = u;
    T.X[r * SD + f] = f2bf(u);
  }
  wave_sync();
  f32x4 q[4], p1[4], p2[4], q3[4], r1[4], r2[4], A3[4], A2[4], A1[4];
  mm<DIM, HID, SD, SD>(T.X, N.W1, q);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a1[ct][v], d, dd);
      p1[ct][v] = q[ct][v] * d;
      r1[ct][v] = q[ct][v] * S.gh1[ct][v] * dd;
    }
  wave_sync();
  put<HID, SH>(T.H, p1);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W2, q);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a2[ct][v], d, dd);
      p2[ct][v] = q[ct][v] * d;
      r2[ct][v] = q[ct][v] * S.gh2[ct][v] * dd;
    }
  wave_sync();
  put<HID, SH>(T.H, p2);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W3, q3);
  float dEm = A.dE[model] * sc;
  float dEr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) dEr[v] = T.rows[rg + v] >= 0 ? dEm : 0.0f;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a3[ct][v], d, dd);
      A3[ct][v] = dEr[v] * S.ga3[ct][v] + q3[ct][v] * N.w4[ct * 16 + c0] * dd;
    }
  wave_sync();
  put<HID, SH>(T.H, A3);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W3T, q);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a2[ct][v], d, dd);
      A2[ct][v] = q[ct][v] * d + r2[ct][v];
    }
  wave_sync();
  put<HID, SH>(T.H, A2);
  wave_sync();
  mm<HID, HID, SH, SH>(T.H, N.W2T, q);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a1[ct][v], d, dd);
      A1[ct][v] = q[ct][v] * d + r1[ct][v];
    }
  float* Gd = A.grad + ((size_t)model * 2 + sp) * NPAR;
  // layer 1: A1^T x + ga1^T un
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) { RA[rg + v][ct * 16 + c0] = A1[ct][v]; RB[rg + v][ct * 16 + c0] = S.ga1[ct][v]; }
  wave_sync();
  for (int k = l; k < HID * DIM; k += WAVE) {
    int o = k / DIM, f = k % DIM;
    float s = 0;
    for (int r = 0; r < 16; ++r) s += RA[r][o] * XN[r][f] + RB[r][o] * UN[r][f];
    if (s != 0) atomicAdd(&Gd[OW1 + k], s);
  }
  {
    float s = 0;
    for (int r = 0; r < 16; ++r) s += RA[r][l];
    if (s != 0) atomicAdd(&Gd[OB1 + l], s);
  }
  wave_sync();
  // layer 2: A2^T h1 + ga2^T p1
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      RA[rg + v][ct * 16 + c0] = A2[ct][v];
      RB[rg + v][ct * 16 + c0] = S.ga2[ct][v];
      RC[rg + v][ct * 16 + c0] = silu(S.a1[ct][v]);
      XN[rg + v][ct * 16 + c0] = p1[ct][v];
    }
  wave_sync();
  for (int k = l; k < HID * HID; k += WAVE) {
    int o = k / HID, f = k % HID;
    float s = 0;
    for (int r = 0; r < 16; ++r) s += RA[r][o] * RC[r][f] + RB[r][o] * XN[r][f];
    if (s != 0) atomicAdd(&Gd[OW2 + k], s);
  }
  {
    float s = 0;
    for (int r = 0; r < 16; ++r) s += RA[r][l];
    if (s != 0) atomicAdd(&Gd[OB2 + l], s);
  }
  wave_sync();
  // layer 3: A3^T h2 + ga3^T p2; output layer dE h3 + s'(a3) q3
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float d, dd;
      silu_d(S.a3[ct][v], d, dd);
      RA[rg + v][ct * 16 + c0] = A3[ct][v];
      RB[rg + v][ct * 16 + c0] = S.ga3[ct][v];
      RC[rg + v][ct * 16 + c0] = silu(S.a2[ct][v]);
      XN[rg + v][ct * 16 + c0] = p2[ct][v];
      UN[rg + v][ct * 16 + c0] = dEr[v] * silu(S.a3[ct][v]) + q3[ct][v] * d;
    }
  wave_sync();
  for (int k = l; k < HID * HID; k += WAVE) {
    int o = k / HID, f = k % HID;
    float s = 0;
    for (int r = 0; r < 16; ++r) s += RA[r][o] * RC[r][f] + RB[r][o] * XN[r][f];
    if (s != 0) atomicAdd(&Gd[OW3 + k], s);
  }
  {
    float s3 = 0, s4 = 0;
    for (int r = 0; r < 16; ++r) { s3 += RA[r][l]; s4 += UN[r][l]; }
    if (s3 != 0) atomicAdd(&Gd[OB3 + l], s3);
    if (s4 != 0) atomicAdd(&Gd[OW4 + l], s4);
  }
  if (l == 0) {
    float s = 0;
    for (int r = 0; r < 16; ++r) s += T.rows[r] >= 0 ? dEm : 0.0f;
    if (s != 0) atomicAdd(&Gd[OB4], s);
  }
}

// Atoms per species and their order ([2][n]); cnt must start at zero.
__global__ void k_order(const Dev D, int* __restrict__ order, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = i < D.n;
  int sp = live && __double2int_rn(D.x[i].w) != 0 ? 1 : 0;   // invalid codes are reported by k_load
  int p0 = wave_append(&cnt[0], live && sp == 0, 1);
  int p1 = wave_append(&cnt[1], live && sp == 1, 1);
  if (live) order[(size_t)sp * D.n + (sp == 0 ? p0 : p1)] = i;
}

// Ensemble: mean force (plus far field) into F, per-atom spread (RMS over
// models of |F_m - mean|), its maximum (float bits), per-model energy sums.
__global__ void k_ens(int n, int nm, const float* __restrict__ Fm, const double* __restrict__ Ff,
                      const float* __restrict__ Em, double* __restrict__ F, float* __restrict__ spread,
                      unsigned* __restrict__ maxbits, double* __restrict__ acc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  float sp = 0;
  double es[NM_MAX] = {0, 0, 0, 0};
  if (i < n) {
    float f[NM_MAX][3] = {};
    float mean[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m)
      if (m < nm) {
        for (int c = 0; c < 3; ++c) { f[m][c] = Fm[((size_t)m * n + i) * 3 + c]; mean[c] += f[m][c]; }
        es[m] = Em[(size_t)m * n + i];
      }
    for (int c = 0; c < 3; ++c) mean[c] /= nm;
    float var = 0;
#pragma unroll
    for (int m = 0; m < NM_MAX; ++m)
      if (m < nm)
        for (int c = 0; c < 3; ++c) var += (f[m][c] - mean[c]) * (f[m][c] - mean[c]);
    sp = sqrtf(var / nm);
    if (spread) spread[i] = sp;
    for (int c = 0; c < 3; ++c) F[3 * i + c] = (double)mean[c] + Ff[3 * i + c];
  }
  float mx = sp;
  for (int o = WAVE / 2; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  int lane = threadIdx.x & (WAVE - 1);
  if (lane == 0 && mx > 0) atomicMax(maxbits, __float_as_uint(mx));
#pragma unroll
  for (int m = 0; m < NM_MAX; ++m)
    if (m < nm) {
      double s = es[m];
      for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0 && s != 0) atomic_add(&acc[(blockIdx.x & (NSLOT - 1)) * N_A + N_E + m], s);
    }
}

// Fold the surrogate's accumulators into the AIREBO context's, so NVE thermo
// rows and the energy output see the surrogate energy, and decide the
// fallback: skip = 1 keeps the surrogate result; skip = 0 lets the AIREBO
// kernels that follow overwrite it.  out (optional): {E_NN mean over models,
// E_far, E_NN spread over models, max force spread, fallback}.
__global__ void k_decide(Dev D, int nm, const double* __restrict__ acc, const unsigned* __restrict__ maxbits,
                         float thr, int* __restrict__ skip, double* __restrict__ out) {
  __shared__ double tot[N_A];
  int t = threadIdx.x;
  if (t < N_A) {
    double s = 0;
    for (int g = 0; g < NSLOT; ++g) s += acc[g * N_A + t];
    tot[t] = s;
  }
  for (int k = t; k < NSLOT * A_N; k += blockDim.x) D.acc[k] = 0;
  __syncthreads();
  if (t == 0) {
    double em = 0, e2 = 0;
    for (int m = 0; m < nm; ++m) em += tot[N_E + m];
    em /= nm;
    for (int m = 0; m < nm; ++m) e2 += (tot[N_E + m] - em) * (tot[N_E + m] - em);
    float mx = __uint_as_float(*maxbits);
    int keep = mx <= thr ? 1 : 0;   // a NaN spread falls back
    *skip = keep;
    D.acc[A_EREBO] = em + tot[N_EFAR];
    for (int c = 0; c < 6; ++c) D.acc[A_VIR + c] = tot[N_VIR + c];
    if (!keep) atomicAdd(&D.stats[S_FALLBACK], 1ull);
    if (!isfinite(em + tot[N_EFAR])) atomicOr(D.flags, F_NONFINITE);
    if (out) {
      out[0] = em; out[1] = tot[N_EFAR]; out[2] = sqrt(e2 / nm); out[3] = mx; out[4] = keep ? 0.0 : 1.0;
    }
  }
}

// Energy output of a surrogate evaluation: total from the context's
// accumulators (surrogate or fallback), the surrogate's parts beside it.
__global__ void k_nn_energy(const double* __restrict__ fin, const double* __restrict__ out, double* __restrict__ energy) {
  if (threadIdx.x == 0) {
    energy[0] = fin[0];
    energy[1] = out[0];
    energy[2] = out[1];
    energy[3] = out[2];
  }
}

// Virial sums of the accumulators (descriptor VJP alone).
__global__ void k_vir_out(const double* __restrict__ acc, double* __restrict__ vir) {
  int c = threadIdx.x;
  if (c >= 6) return;
  double s = 0;
  for (int g = 0; g < NSLOT; ++g) s += acc[g * N_A + N_VIR + c];
  vir[c] = s;
}

// Training residuals: Wres[m][i] = -2 wF (F_m,i - (Fref_i - Ffar_i)); force
// loss wF |.|^2 summed per model into acc[N_LOSSF + m].
__global__ void k_residual(int n, int nm, const float* __restrict__ Fm, const double* __restrict__ Fref,
                           const double* __restrict__ Ff, double wF, float* __restrict__ Wres,
                           double* __restrict__ acc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double lf[NM_MAX] = {0, 0, 0, 0};
#pragma unroll
  for (int m = 0; m < NM_MAX; ++m)
    if (m < nm && i < n)
      for (int c = 0; c < 3; ++c) {
        double d = (double)Fm[((size_t)m * n + i) * 3 + c] - (Fref[3 * i + c] - Ff[3 * i + c]);
        Wres[((size_t)m * n + i) * 3 + c] = (float)(-2.0 * wF * d);
        lf[m] += wF * d * d;
      }
  int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
  for (int m = 0; m < NM_MAX; ++m)
    if (m < nm) {
      double s = lf[m];
      for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0 && s != 0) atomic_add(&acc[(blockIdx.x & (NSLOT - 1)) * N_A + N_LOSSF + m], s);
    }
}

// Energy adjoint per model, dE[m] = 2 wE (E_m + E_far - E_ref), and loss[m] =
// force loss + wE (E_m + E_far - E_ref)^2.
__global__ void k_energy_seed(int nm, const double* __restrict__ acc, double eref, double wE, float* __restrict__ dE,
                              double* __restrict__ loss) {
  int m = threadIdx.x;
  if (m >= nm) return;
  double em = 0, ef = 0, lf = 0;
  for (int g = 0; g < NSLOT; ++g) {
    em += acc[g * N_A + N_E + m];
    ef += acc[g * N_A + N_EFAR];
    lf += acc[g * N_A + N_LOSSF + m];
  }
  double d = em + ef - eref;
  dE[m] = (float)(2.0 * wE * d);
  loss[m] = lf + wE * d * d;
}

__global__ void k_fill(float* __restrict__ p, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = 0.0f;
}
__global__ void k_fill_d(double* __restrict__ p, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) p[k] = 0.0;
}
__global__ void k_zero_small(int* __restrict__ cnt, unsigned* __restrict__ maxbits) {
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) *maxbits = 0;
}

// Adam on FP32 parameters (bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t).
__global__ void k_adam(int np, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  float gv = g[k];
  float a = b1 * m1[k] + (1.0f - b1) * gv;
  float b = b2 * m2[k] + (1.0f - b2) * gv * gv;
  m1[k] = a;
  m2[k] = b;
  p[k] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// Column sums and sums of squares of G [rows][DIM] into mom[2][DIM].
__global__ void k_moments(const float* __restrict__ G, int64_t rows, double* __restrict__ mom) {
  int f = threadIdx.x;
  if (f >= DIM) return;
  double s = 0, s2 = 0;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    double v = G[r * DIM + f];
    s += v;
    s2 += v * v;
  }
  atomic_add(&mom[f], s);
  atomic_add(&mom[DIM + f], s2);
}

}  // namespace nn
}  // namespace airebo

// ---------------------------------------------------------------------------
// Host side of the surrogate
// ---------------------------------------------------------------------------
using namespace airebo::nn;

struct airebo_nn {
  int nm = 0;
  int device = 0;
  float* params = nullptr;   // [nm][2][NPAR]
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  int64_t adam_t = 0;
  float* mean = nullptr;     // [DIM]
  float* istd = nullptr;     // [DIM]
  float* shift = nullptr;    // [2]
  float scale = 1.0f;
  std::vector<float> h_mean, h_istd;
  float h_shift[2] = {0, 0};
  float *G = nullptr, *dEdG = nullptr, *U = nullptr, *Eat = nullptr, *Fm = nullptr, *Wres = nullptr,
        *spread = nullptr, *dE = nullptr;
  size_t cG = 0, cdg = 0, cU = 0, cE = 0, cFm = 0, cW = 0, csp = 0, cdE = 0;
  double *Ff = nullptr, *acc = nullptr, *out = nullptr, *loss = nullptr, *mom = nullptr, *fin = nullptr,
         *vir = nullptr;
  size_t cFf = 0, cacc = 0, cout = 0, closs = 0, cmom = 0, cfin = 0, cvir = 0;
  int *order = nullptr, *cnt = nullptr, *skip = nullptr;
  size_t cord = 0, ccnt = 0, cskip = 0;
  unsigned* maxbits = nullptr;
  size_t cmax = 0;
  NetLDS* packed = nullptr;   // [nm][2] BF16 images for inference
  bool stale = true;          // images out of date after a weight update
};

namespace {

int nn_buffers(airebo_nn* m, int64_t n, bool train) {
  size_t N = (size_t)std::max<int64_t>(n, 1);
  int rc = 0;
  rc |= grow(m->G, m->cG, N * DIM);
  rc |= grow(m->dEdG, m->cdg, (size_t)m->nm * N * DIM);
  rc |= grow(m->Eat, m->cE, (size_t)m->nm * N);
  rc |= grow(m->Fm, m->cFm, (size_t)m->nm * N * 3);
  rc |= grow(m->spread, m->csp, N);
  rc |= grow(m->Ff, m->cFf, N * 3);
  rc |= grow(m->acc, m->cacc, (size_t)NSLOT * N_A);
  rc |= grow(m->out, m->cout, 8);
  rc |= grow(m->fin, m->cfin, 8);
  rc |= grow(m->vir, m->cvir, 8);
  rc |= grow(m->order, m->cord, 2 * N);
  rc |= grow(m->cnt, m->ccnt, 2);
  rc |= grow(m->skip, m->cskip, 1);
  rc |= grow(m->maxbits, m->cmax, 1);
  rc |= grow(m->dE, m->cdE, NM_MAX);
  rc |= grow(m->loss, m->closs, NM_MAX);
  rc |= grow(m->mom, m->cmom, 2 * DIM);
  if (train) {
    rc |= grow(m->U, m->cU, (size_t)m->nm * N * DIM);
    rc |= grow(m->Wres, m->cW, (size_t)m->nm * N * 3);
  }
  return rc ? AIREBO_E_DEVICE : 0;
}

NNArgs nn_args(airebo_nn* m, int n) {
  NNArgs a;
  std::memset(&a, 0, sizeof a);
  a.n = n;
  a.order = m->order;
  a.cnt = m->cnt;
  a.G = m->G;
  a.mean = m->mean;
  a.istd = m->istd;
  a.params = m->params;
  a.scale = m->scale;
  a.shift = m->shift;
  a.E = m->Eat;
  a.dEdG = m->dEdG;
  a.U = m->U;
  a.dE = m->dE;
  a.grad = m->grad;
  return a;
}

// Descriptors and networks of all models on the context's current positions
// and lists (G, per-atom energies, dE/dG), then the descriptor VJP into the
// per-model forces and the far field.
void nn_core(airebo_ctx* c, airebo_nn* m, hipStream_t s) {
  Dev& D = c->D;
  int n = D.n;
  size_t nF = (size_t)m->nm * n * 3;
  LAUNCH(c, K_NN_ZERO, k_fill, dim3(std::min<int64_t>(blocks((int64_t)nF, 256), 4096)), dim3(256), s, m->Fm, nF);
  LAUNCH(c, K_NN_ZERO, k_fill_d, dim3(blocks(NSLOT * N_A, 256)), dim3(256), s, m->acc, (size_t)NSLOT * N_A);
  LAUNCH(c, K_NN_ZERO, k_zero_small, dim3(1), dim3(64), s, m->cnt, m->maxbits);
  LAUNCH(c, K_NN_ORDER, k_order, dim3(blocks(n, 256)), dim3(256), s, D, m->order, m->cnt);
  LAUNCH(c, K_NN_DESC, k_desc<0>, dim3(blocks((int64_t)n * WAVE, 256)), dim3(256), s, D, m->G, (const float*)nullptr);
  if (m->stale) {
    LAUNCH(c, K_NN_PACK, k_pack, dim3(2 * m->nm), dim3(256), s, (const float*)m->params, m->packed);
    m->stale = false;
  }
  NNArgs a = nn_args(m, n);
  int gx = std::max(1, std::min(blocks(blocks(n, 16), 2 * MLP_WAVES), 256));
  LAUNCH(c, K_NN_MLP, k_mlp, dim3(gx, 2 * m->nm), dim3(64 * MLP_WAVES), s, a, (const NetLDS*)m->packed);
  LAUNCH(c, K_NN_FORCE, k_desc_force<true>, dim3(n), dim3(WAVE), s, D,
         (const DevParams*)c->dP, (const float*)m->dEdG, m->nm, m->Fm, m->Ff, m->acc);
  LAUNCH(c, K_NN_ENS, k_ens, dim3(blocks(n, 256)), dim3(256), s, n, m->nm, (const float*)m->Fm, (const double*)m->Ff,
         (const float*)m->Eat, D.F, m->spread, m->maxbits, m->acc);
}

// The surrogate's full force step: core, ensemble decision, then the AIREBO
// force kernels, which run only when the decision asks for the fallback.
void nn_step(airebo_ctx* c, airebo_nn* m, float thr, hipStream_t s) {
  nn_core(c, m, s);
  LAUNCH(c, K_NN_DECIDE, k_decide, dim3(1), dim3(256), s, c->D, m->nm, (const double*)m->acc,
         (const unsigned*)m->maxbits, thr, m->skip, m->out);
  launch_forces(c, s);
}

int nn_check(airebo_nn* m) {
  if (!m || m->nm < 1) return fail(AIREBO_E_ARG, "null surrogate");
  return 0;
}

int nn_args_ok(airebo_ctx* c, int64_t n, const double* pos, const int32_t* species, const double* box,
               const int32_t* periodic) {
  if (!c || !box || !periodic || !pos || !species) return fail(AIREBO_E_ARG, "null argument");
  if (n < 1 || n >= (1ll << 27)) return fail(AIREBO_E_ARG, "n out of range");
  return 0;
}

// Positions into the context and lists rebuilt (LJ capacity grown and the
// evaluation repeated when it overflows), then `body` launched; flags checked.
template <typename Body>
int nn_eval(airebo_ctx* c, int64_t n, const double* pos, const int32_t* species, const double* box,
            const int32_t* periodic, hipStream_t s, Body body) {
  HIPCHK(hipSetDevice(c->opt.device));
  c->regrow = 0;
  int64_t off[2] = {0, n};
  for (int attempt = 0; attempt < 4; ++attempt) {
    int rc = setup(c, 1, off, box, periodic, s);
    if (rc) return rc;
    Dev& D = c->D;
    D.F = c->F;
    HIPCHK(hipMemsetAsync(c->stats, 0, S_N * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_set_flags, dim3(1), dim3(64), 0, s, D, F_REBUILD);
    HIPCHK(hipMemsetAsync(c->cell_count, 0, sizeof(int) * c->ncell, s));
    hipLaunchKernelGGL(k_load, dim3(blocks(n, 256)), dim3(256), 0, s, D, pos, species, 0);
    launch_rebuild(c, s);
    int g = std::min(blocks(n, 256), 1024);
    hipLaunchKernelGGL(k_max, dim3(g), dim3(256), 0, s, (const int*)D.lj_n, (int)n, D.lj_cap, D.stats + S_MAXLJ,
                       D.stats + S_LJENT, (unsigned long long*)nullptr);
    hipLaunchKernelGGL(k_max, dim3(g), dim3(256), 0, s, (const int*)D.lf_n, (int)n, D.lf_cap, D.stats + S_MAXLF,
                       D.stats + S_LJENT, D.stats + S_LFENT);
    rc = body(D);
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    int flags = 0;
    HIPCHK(hipMemcpyAsync(&flags, c->flags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(c->host_stats, c->stats, sizeof c->host_stats, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if ((flags & F_GROW) && !(flags & (F_BADSPEC | F_NONFINITE))) {
      if (grow_caps(c, flags)) return check_flags(c, flags);
      continue;
    }
    return check_flags(c, flags);
  }
  return fail(AIREBO_E_CAPACITY, "list or queue capacity could not be established");
}

const char kMagic[8] = {'A', 'I', 'R', 'N', 'N', '0', '0', '1'};

}  // namespace

extern "C" {

int airebo_nn_create(int32_t nmodels, int32_t device, airebo_nn_t* out) {
  if (!out || nmodels < 1 || nmodels > NM_MAX) return fail(AIREBO_E_ARG, "models must be 1..4");
  HIPCHK(hipSetDevice(device));
  airebo_nn* m = new airebo_nn();
  m->nm = nmodels;
  m->device = device;
  size_t np = (size_t)nmodels * 2 * NPAR;
  size_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0;
  int rc = 0;
  rc |= grow(m->params, c0, np);
  rc |= grow(m->grad, c1, np);
  rc |= grow(m->m1, c2, np);
  rc |= grow(m->m2, c3, np);
  rc |= grow(m->mean, c4, DIM);
  rc |= grow(m->istd, c5, DIM);
  rc |= grow(m->shift, c6, 2);
  size_t c7 = 0;
  rc |= grow(m->packed, c7, (size_t)nmodels * 2);
  if (rc) { airebo_nn_free(m); return AIREBO_E_DEVICE; }
  m->h_mean.assign(DIM, 0.0f);
  m->h_istd.assign(DIM, 1.0f);
  std::vector<float> zeros(np, 0.0f);
  hipError_t e = hipMemcpy(m->params, zeros.data(), np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m1, zeros.data(), np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m2, zeros.data(), np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->grad, zeros.data(), np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->mean, m->h_mean.data(), DIM * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->istd, m->h_istd.data(), DIM * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->shift, m->h_shift, 2 * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    std::string msg = hipGetErrorString(e);
    airebo_nn_free(m);
    return fail(AIREBO_E_DEVICE, msg);
  }
  *out = m;
  return 0;
}

void airebo_nn_free(airebo_nn_t m) {
  if (!m) return;
  void* ptrs[] = {m->params, m->grad, m->m1, m->m2, m->mean, m->istd, m->shift, m->G, m->dEdG, m->U, m->Eat,
                  m->Fm, m->Wres, m->spread, m->dE, m->Ff, m->acc, m->out, m->loss, m->mom, m->fin, m->vir,
                  m->order, m->cnt, m->skip, m->maxbits, m->packed};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

int airebo_nn_sizes(int32_t* dim, int32_t* params_per_net) {
  if (!dim || !params_per_net) return fail(AIREBO_E_ARG, "null argument");
  *dim = DIM;
  *params_per_net = NPAR;
  return 0;
}

int airebo_nn_models(airebo_nn_t m) { return m ? m->nm : 0; }

int airebo_nn_set_params(airebo_nn_t m, const float* host) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!host) return fail(AIREBO_E_ARG, "null argument");
  size_t np = (size_t)m->nm * 2 * NPAR;
  for (size_t k = 0; k < np; ++k)
    if (!std::isfinite(host[k])) return fail(AIREBO_E_ARG, "non-finite weight");
  HIPCHK(hipSetDevice(m->device));
  HIPCHK(hipMemcpy(m->params, host, sizeof(float) * np, hipMemcpyHostToDevice));
  m->stale = true;
  m->adam_t = 0;
  std::vector<float> zeros(np, 0.0f);
  HIPCHK(hipMemcpy(m->m1, zeros.data(), np * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(m->m2, zeros.data(), np * 4, hipMemcpyHostToDevice));
  return 0;
}

int airebo_nn_get_params(airebo_nn_t m, float* host) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!host) return fail(AIREBO_E_ARG, "null argument");
  HIPCHK(hipSetDevice(m->device));
  HIPCHK(hipMemcpy(host, m->params, sizeof(float) * m->nm * 2 * NPAR, hipMemcpyDeviceToHost));
  return 0;
}

int airebo_nn_get_grad(airebo_nn_t m, float* host) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!host) return fail(AIREBO_E_ARG, "null argument");
  HIPCHK(hipSetDevice(m->device));
  HIPCHK(hipMemcpy(host, m->grad, sizeof(float) * m->nm * 2 * NPAR, hipMemcpyDeviceToHost));
  return 0;
}

int airebo_nn_set_norm(airebo_nn_t m, const float* mean, const float* istd, double scale, const double* shift) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!mean || !istd || !shift) return fail(AIREBO_E_ARG, "null argument");
  if (!(scale > 0) || !std::isfinite(scale) || !std::isfinite(shift[0]) || !std::isfinite(shift[1]))
    return fail(AIREBO_E_ARG, "scale must be positive and shifts finite");
  for (int f = 0; f < DIM; ++f)
    if (!std::isfinite(mean[f]) || !(istd[f] > 0) || !std::isfinite(istd[f]))
      return fail(AIREBO_E_ARG, "normalisation must be finite with positive inverse deviations");
  HIPCHK(hipSetDevice(m->device));
  m->h_mean.assign(mean, mean + DIM);
  m->h_istd.assign(istd, istd + DIM);
  m->scale = (float)scale;
  m->h_shift[0] = (float)shift[0];
  m->h_shift[1] = (float)shift[1];
  HIPCHK(hipMemcpy(m->mean, mean, DIM * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(m->istd, istd, DIM * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(m->shift, m->h_shift, 2 * 4, hipMemcpyHostToDevice));
  return 0;
}

int airebo_nn_get_norm(airebo_nn_t m, float* mean, float* istd, double* scale, double* shift) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!mean || !istd || !scale || !shift) return fail(AIREBO_E_ARG, "null argument");
  std::memcpy(mean, m->h_mean.data(), DIM * 4);
  std::memcpy(istd, m->h_istd.data(), DIM * 4);
  *scale = m->scale;
  shift[0] = m->h_shift[0];
  shift[1] = m->h_shift[1];
  return 0;
}

int airebo_nn_moments(airebo_nn_t m, const float* G, int64_t rows, double* mom_host, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!G || !mom_host || rows < 1) return fail(AIREBO_E_ARG, "null argument or no rows");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipSetDevice(m->device));
  int rc = nn_buffers(m, 1, false);
  if (rc) return rc;
  hipLaunchKernelGGL(k_fill_d, dim3(1), dim3(256), 0, s, m->mom, (size_t)2 * DIM);
  hipLaunchKernelGGL(k_moments, dim3((unsigned)std::min<int64_t>(rows, 2048)), dim3(128), 0, s, G, rows, m->mom);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(mom_host, m->mom, sizeof(double) * 2 * DIM, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return 0;
}

int airebo_nn_descriptors(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                          const double* box, const int32_t* periodic, float* G, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!G) return fail(AIREBO_E_ARG, "null argument");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  return nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
    hipLaunchKernelGGL(k_desc<0>, dim3(blocks((int64_t)n * WAVE, 256)), dim3(256), 0, s, D, G, (const float*)nullptr);
    return 0;
  });
}

int airebo_nn_descriptor_jvp(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                             const double* box, const int32_t* periodic, const float* w, float* out, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!w || !out) return fail(AIREBO_E_ARG, "null argument");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  return nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
    hipLaunchKernelGGL(k_desc<1>, dim3(blocks((int64_t)n * WAVE, 256)), dim3(256), 0, s, D, out, w);
    return 0;
  });
}

int airebo_nn_descriptor_vjp(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                             const double* box, const int32_t* periodic, const float* g, int32_t nsets, float* F,
                             double* virial, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!g || !F || !virial) return fail(AIREBO_E_ARG, "null argument");
  if (nsets < 1 || nsets > NM_MAX) return fail(AIREBO_E_ARG, "nsets must be 1..4");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  rc = nn_buffers(m, n, false);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  return nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
    size_t nF = (size_t)nsets * n * 3;
    hipLaunchKernelGGL(k_fill, dim3(std::min<int64_t>(blocks((int64_t)nF, 256), 4096)), dim3(256), 0, s, F, nF);
    hipLaunchKernelGGL(k_fill_d, dim3(blocks(NSLOT * N_A, 256)), dim3(256), 0, s, m->acc, (size_t)NSLOT * N_A);
    hipLaunchKernelGGL(k_desc_force<false>, dim3(n), dim3(WAVE), 0, s, D,
                       (const DevParams*)c->dP, g, (int)nsets, F, (double*)nullptr, m->acc);
    hipLaunchKernelGGL(k_vir_out, dim3(1), dim3(64), 0, s, (const double*)m->acc, virial);
    return 0;
  });
}

int airebo_nn_compute(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                      const double* box, const int32_t* periodic, double threshold, double* energy, double* forces,
                      double* virial, float* spread, double* info, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!energy || !forces || !virial) return fail(AIREBO_E_ARG, "null argument");
  if (!(threshold > 0)) return fail(AIREBO_E_ARG, "threshold must be positive");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  if (c->opt.device != m->device) return fail(AIREBO_E_ARG, "context and surrogate on different devices");
  rc = nn_buffers(m, n, false);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  float thr = (float)std::min(threshold, 1e30);
  rc = nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
    D.F = forces;
    D.skip = m->skip;
    nn_step(c, m, thr, s);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(256), 0, s, D, m->fin, virial);
    hipLaunchKernelGGL(k_nn_energy, dim3(1), dim3(64), 0, s, (const double*)m->fin, (const double*)m->out, energy);
    if (spread) HIPCHK(hipMemcpyAsync(spread, m->spread, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    if (info) HIPCHK(hipMemcpyAsync(info, m->out, sizeof(double) * 5, hipMemcpyDeviceToHost, s));
    return 0;
  });
  c->D.skip = nullptr;
  return rc;
}

int airebo_nn_gradient(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                       const double* box, const int32_t* periodic, const double* f_ref, double e_ref, double w_force,
                       double w_energy, double* loss, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!f_ref || !loss) return fail(AIREBO_E_ARG, "null argument");
  if (!(w_force >= 0) || !(w_energy >= 0) || !std::isfinite(e_ref)) return fail(AIREBO_E_ARG, "bad loss weights");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  if (c->opt.device != m->device) return fail(AIREBO_E_ARG, "context and surrogate on different devices");
  rc = nn_buffers(m, n, true);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  return nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
    nn_core(c, m, s);
    int nn = (int)n;
    hipLaunchKernelGGL(k_residual, dim3(blocks(n, 256)), dim3(256), 0, s, nn, m->nm, (const float*)m->Fm, f_ref,
                       (const double*)m->Ff, w_force, m->Wres, m->acc);
    hipLaunchKernelGGL(k_energy_seed, dim3(1), dim3(64), 0, s, m->nm, (const double*)m->acc, e_ref, w_energy, m->dE,
                       m->loss);
    for (int k = 0; k < m->nm; ++k)
      hipLaunchKernelGGL(k_desc<1>, dim3(blocks((int64_t)n * WAVE, 256)), dim3(256), 0, s, D,
                         m->U + (size_t)k * n * DIM, (const float*)(m->Wres + (size_t)k * n * 3));
    size_t np = (size_t)m->nm * 2 * NPAR;
    hipLaunchKernelGGL(k_fill, dim3(blocks((int64_t)np, 256)), dim3(256), 0, s, m->grad, np);
    NNArgs a = nn_args(m, nn);
    hipLaunchKernelGGL(k_mlp_train, dim3(blocks(n, 16) + 1, m->nm), dim3(64), 0, s, a);
    HIPCHK(hipMemcpyAsync(loss, m->loss, sizeof(double) * m->nm, hipMemcpyDeviceToHost, s));
    return 0;
  });
}

int airebo_nn_adam(airebo_nn_t m, double lr, double beta1, double beta2, double eps, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(AIREBO_E_ARG, "bad Adam settings");
  HIPCHK(hipSetDevice(m->device));
  m->adam_t += 1;
  double c1 = 1.0 - std::pow(beta1, (double)m->adam_t), c2 = 1.0 - std::pow(beta2, (double)m->adam_t);
  int np = m->nm * 2 * NPAR;
  hipLaunchKernelGGL(k_adam, dim3(blocks(np, 256)), dim3(256), 0, (hipStream_t)stream, np, m->params,
                     (const float*)m->grad, m->m1, m->m2, (float)lr, (float)beta1, (float)beta2, (float)eps,
                     (float)c1, (float)c2);
  HIPCHK(hipGetLastError());
  m->stale = true;
  return 0;
}

int airebo_nn_train_step(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const int32_t* species,
                         const double* box, const int32_t* periodic, const double* f_ref, double e_ref,
                         double w_force, double w_energy, double lr, double* loss, void* stream) {
  int rc = airebo_nn_gradient(m, c, n, pos, species, box, periodic, f_ref, e_ref, w_force, w_energy, loss, stream);
  if (rc) return rc;
  return airebo_nn_adam(m, lr, 0.9, 0.999, 1e-8, stream);
}

int airebo_nn_md_begin(airebo_nn_t m, airebo_ctx_t c, int64_t n, const double* pos, const double* vel,
                       const int32_t* species, const double* box, const int32_t* periodic, const double* mass,
                       double dt, double threshold, void* stream) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!vel || !mass) return fail(AIREBO_E_ARG, "null argument");
  int rc = nn_args_ok(c, n, pos, species, box, periodic);
  if (rc) return rc;
  if (!(dt > 0) || !(mass[0] > 0) || !(mass[1] > 0) || !(threshold > 0))
    return fail(AIREBO_E_ARG, "bad dt, mass or threshold");
  if (c->opt.device != m->device) return fail(AIREBO_E_ARG, "context and surrogate on different devices");
  rc = nn_buffers(m, n, false);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  float thr = (float)std::min(threshold, 1e30);
  auto size = [&]() -> int {   // list capacity from a plain surrogate evaluation
    int r = nn_eval(c, n, pos, species, box, periodic, s, [&](Dev& D) -> int {
      D.skip = m->skip;
      nn_step(c, m, thr, s);
      return 0;
    });
    c->D.skip = nullptr;
    return r;
  };
  int64_t off[2] = {0, n};
  return md_begin_impl(c, 1, off, box, periodic, pos, vel, species, mass, dt, s, size,
                       [c, m, thr](hipStream_t st, bool) { nn_step(c, m, thr, st); }, m->skip);
}

int airebo_nn_nve(airebo_nn_t m, airebo_ctx_t c, int64_t n, double* pos, double* vel, const int32_t* species,
                  const double* box, const int32_t* periodic, const double* mass, double dt, int64_t nsteps,
                  int64_t every, double* thermo, double threshold, int64_t* fallbacks, void* stream) {
  if (nsteps < 0) return fail(AIREBO_E_ARG, "bad step count");
  if (every > 0 && !thermo) return fail(AIREBO_E_ARG, "thermo output needed when thermo_every > 0");
  hipStream_t s = (hipStream_t)stream;
  int rc = airebo_nn_md_begin(m, c, n, pos, vel, species, box, periodic, mass, dt, threshold, stream);
  if (!rc) rc = md_run_impl(c, nsteps, every, thermo, s);
  int rc2 = c && c->md.on ? md_state_impl(c, pos, vel, s) : 0;
  if (c && c->md.on) {
    hipError_t e = hipStreamSynchronize(s);
    if (!rc2 && e != hipSuccess) rc2 = fail(AIREBO_E_DEVICE, std::string("surrogate nve: ") + hipGetErrorString(e));
  }
  if (c) md_end_impl(c);
  if (!rc && fallbacks) *fallbacks = (int64_t)c->host_stats[S_FALLBACK];
  return rc ? rc : rc2;
}

int airebo_nn_profile_nve(airebo_nn_t m, airebo_ctx_t c, int64_t n, double* pos, double* vel,
                          const int32_t* species, const double* box, const int32_t* periodic, const double* mass,
                          double dt, int64_t nsteps, double threshold, double* ms_out, int64_t* launches_out,
                          void* stream) {
  if (!c || !ms_out || !launches_out) return fail(AIREBO_E_ARG, "null argument");
  c->prof = true;
  c->ev.clear();
  int rc = airebo_nn_nve(m, c, n, pos, vel, species, box, periodic, mass, dt, nsteps, 0, nullptr, threshold,
                         nullptr, stream);
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

int airebo_nn_save(airebo_nn_t m, const char* path) {
  if (nn_check(m)) return AIREBO_E_ARG;
  if (!path) return fail(AIREBO_E_ARG, "null argument");
  std::vector<float> p((size_t)m->nm * 2 * NPAR);
  int rc = airebo_nn_get_params(m, p.data());
  if (rc) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(AIREBO_E_ARG, std::string("cannot write ") + path);
  int32_t hdr[3] = {m->nm, DIM, NPAR};
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 3, f) == 3 &&
            std::fwrite(&m->scale, 4, 1, f) == 1 && std::fwrite(m->h_shift, 4, 2, f) == 2 &&
            std::fwrite(m->h_mean.data(), 4, DIM, f) == (size_t)DIM &&
            std::fwrite(m->h_istd.data(), 4, DIM, f) == (size_t)DIM &&
            std::fwrite(p.data(), 4, p.size(), f) == p.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? 0 : fail(AIREBO_E_ARG, std::string("write failed: ") + path);
}

int airebo_nn_load(const char* path, int32_t device, airebo_nn_t* out) {
  if (!path || !out) return fail(AIREBO_E_ARG, "null argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(AIREBO_E_ARG, std::string("cannot read ") + path);
  char magic[8];
  int32_t hdr[3];
  float scale, shift[2];
  std::vector<float> mean(DIM), istd(DIM);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(hdr, 4, 3, f) == 3 &&
            hdr[0] >= 1 && hdr[0] <= NM_MAX && hdr[1] == DIM && hdr[2] == NPAR && std::fread(&scale, 4, 1, f) == 1 &&
            std::fread(shift, 4, 2, f) == 2 && std::fread(mean.data(), 4, DIM, f) == (size_t)DIM &&
            std::fread(istd.data(), 4, DIM, f) == (size_t)DIM;
  std::vector<float> p;
  if (ok) {
    p.resize((size_t)hdr[0] * 2 * NPAR);
    ok = std::fread(p.data(), 4, p.size(), f) == p.size();
  }
  std::fclose(f);
  if (!ok) return fail(AIREBO_E_ARG, std::string("not a surrogate file of this layout: ") + path);
  airebo_nn_t m = nullptr;
  int rc = airebo_nn_create(hdr[0], device, &m);
  if (rc) return rc;
  double sh[2] = {shift[0], shift[1]};
  rc = airebo_nn_set_norm(m, mean.data(), istd.data(), scale, sh);
  if (!rc) rc = airebo_nn_set_params(m, p.data());
  if (rc) { airebo_nn_free(m); return rc; }
  *out = m;
  return 0;
}

int airebo_nn_mfma_check(const float* A, const float* B, float* Dout, void* stream) {
  if (!A || !B || !Dout) return fail(AIREBO_E_ARG, "null argument");
  hipLaunchKernelGGL(k_mfma_check, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, Dout);
  HIPCHK(hipGetLastError());
  return 0;
}

int airebo_nn_mfma32_check(const float* A, const float* B, float* Dout, void* stream) {
  if (!A || !B || !Dout) return fail(AIREBO_E_ARG, "null argument");
  hipLaunchKernelGGL(k_mfma32_check, dim3(1), dim3(64), 0, (hipStream_t)stream, A, B, Dout);
  HIPCHK(hipGetLastError());
  return 0;
}

}  // extern "C"
