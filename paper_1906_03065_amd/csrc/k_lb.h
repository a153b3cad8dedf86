// k_lb.h -- the fused lattice-Boltzmann step (Sec. 3.1) for D2Q9.
//
// One kernel does, per node and time step: pull-streaming of f, g, h, the
// moments of eq. MomentsDFs, the Laplacians of rho, phi, psi, the chemical
// potentials of Appendix A (with the coupling term of Sec. 3.1), their
// gradients, the force of eqs. ForcingTermLBE / ForceFE plus the spread
// membrane force, the velocities of eqs. ActualFluidVel / VelCorrection and
// the BGK + exact-difference collision of eq. LBE, writing the post-collision
// populations.  Populations are read once and written once per step.
//
// Dependency chain: the collision at row c needs grad mu at c, i.e. mu on
// rows c-1..c+1, i.e. moments on rows c-2..c+2.  A workgroup owns a strip of
// BX-4 interior columns (BX lanes, two halo columns each side) and marches
// along a segment of rows (up or down) with a three-stage software pipeline:
//   iteration k:  M  pull row r into registers, moments -> LDS ring
//                 U  mu on the previous row from the moment ring -> LDS ring
//                 C  collide the row before that with the populations pulled
//                    two iterations earlier (still in registers) and store.
// Halo columns are recomputed by the neighbouring strip; halo rows only at
// segment ends.  Registers hold three rows of populations; the loop is
// unrolled by three so every register index is a compile-time constant.
//
// Precision: moving populations and their collision use the storage's real
// type R (FP32 or FP64).  Moments, chemical potentials, their stencils and
// the force are FP64: the chemical potential is a sum of terms much larger
// than itself near interfaces, and its Laplacian/gradient chain would turn
// single-precision rounding of phi and psi into force noise.
#pragma once
#include <type_traits>

#include "common.h"
#include "store.h"

namespace lb {

struct LBParams {
  double inv_tau, inv_tau_phi, inv_tau_psi;  // 1/tau (eq. RelaxationTimes)
  double gphi, gpsi;                         // Gamma_phi, Gamma_psi (eq. EDF)
  double k1, k2, k3, a2, kc;                 // kappa_m, alpha^2, kappa_c
  double fext[3];                            // uniform external force density (eq. ForcingTermLBE)
  // component densities M_m (eq. MassDensity; all 1 in the paper): the
  // concentrations are C_m = sum_q cm[m][q] q with q = (rho, phi, psi), and
  // the lattice pressure is c_s^2 (rho + sp) with sp = -(psh[0] phi + psh[1] psi)
  double cm[3][3];
  double psh[2];
  double mb;                                 // (M_1 + M_2) / 2
  // reference density of the stored populations: a kernel holds f_i - w_i rho0
  // (rho0 = M_b, 1 for equal densities), so that the moving populations stay
  // small where the lattice pressure is c_s^2 M_b n with n ~ 1
  double rho0;
  int dens;                                  // 1 if some M_m differs from 1
  int nx, ny, nz, wall_y, wall_z;
  long long N;
  int ntx, nty, tile;                        // tile grid of the membrane maps (edge a power of two)
  int seg;                                   // rows (2D) or planes (3D) per workgroup
  int nstrip, nseg;                          // workgroup grid: strips x segments
  int nxcd;                                  // XCDs the dispatcher deals workgroups to
  int mode;                                  // 2D pass: 0 all, 1 regions without active tiles,
                                             // 2 regions with active tiles (in pieces)
  int seg2, npiece;                          // pass 2: rows per piece, pieces per segment
};

// Workgroup -> (strip, segment).  The dispatcher deals consecutive
// workgroups to the XCDs in turn, and each XCD has its own L2.  Give every
// XCD a contiguous run of the logical order (strips fastest), so the strips
// that share halo columns run side by side on one XCD and meet in its L2.
__device__ __forceinline__ int dealt_index(int b, int total, int nxcd) {
  const int c = b % nxcd, j = b / nxcd;
  // blocks dealt to XCDs before c: sum over c' < c of ceil((total - c') / nxcd)
  const int q = total / nxcd, rem = total % nxcd;
  return c * q + min(c, rem) + j;
}

__device__ __forceinline__ void strip_segment(int b, int nstrip, int nseg, int nxcd, int& s, int& g) {
  const int L = dealt_index(b, nstrip * nseg, nxcd);
  s = L % nstrip;
  g = L / nstrip;
}

// mu_rho (without the ideal-gas part), mu_phi, mu_psi' from local values and
// Laplacians, written through the concentrations C_m, a linear map of
// (rho, phi, psi) (eq. VariableTransform; with component densities, eq.
// MassDensity solved for C_1 + C_2).  The derivative of the Landau energy
// (eq. LandauFE) with respect to C_m is
// b_m = kappa_m C_m (1-C_m)(1-2C_m) - alpha^2 kappa_m lap C_m, and the chain
// rule gives mu_q = sum_m (dC_m/dq) b_m; for equal densities
// mu_rho = (b1+b2)/2, mu_phi = (b1-b2)/2, mu_psi = b3 - (b1+b2)/2.  The
// coupling energy (eq. CouplingE) adds kappa_c (psi - I) to mu_psi.  The
// map's coefficients for equal densities are 0, +-1/2 and 1, so the sums
// round as the closed forms do.
__device__ __forceinline__ void conc3(const LBParams& P, double a, double b, double c, double* C) {
#pragma unroll
  for (int m = 0; m < 3; m++) C[m] = P.cm[m][0] * a + P.cm[m][1] * b + P.cm[m][2] * c;
}

__device__ __forceinline__ void chem_pot(const LBParams& P, double drho, double phi, double psi,
                                         double lr, double lp, double ls, double I, double& mr,
                                         double& mp, double& ms) {
  const double rho = P.rho0 + drho;
  double C[3], Lc[3];
  conc3(P, rho, phi, psi, C);
  conc3(P, lr, lp, ls, Lc);
  const double km[3] = {P.k1, P.k2, P.k3};
  double b[3];
#pragma unroll
  for (int m = 0; m < 3; m++) b[m] = km[m] * (C[m] * (1.0 - C[m]) * (1.0 - 2.0 * C[m]) - P.a2 * Lc[m]);
  mr = (P.cm[0][0] * b[0] + P.cm[1][0] * b[1]) + P.cm[2][0] * b[2];
  mp = (P.cm[0][1] * b[0] + P.cm[1][1] * b[1]) + P.cm[2][1] * b[2];
  ms = (P.cm[0][2] * b[0] + P.cm[1][2] * b[1]) + P.cm[2][2] * b[2] + P.kc * (psi - I);
}

// BGK + exact-difference collision of one node, D2Q9, in place.  pf holds
// f_i - w_i rho0 (all i), pg/ph the moving g_i/h_i (i >= 1), g0/h0 the rest
// populations.  Moments and the total force (Fx, Fy) are FP64.
template <typename R>
__device__ __forceinline__ void collide9(const LBParams& P, R* pf, R* pg, R* ph, double& g0,
                                         double& h0, double drho, double jx, double jy, double phi,
                                         double psi, double mphi, double mpsi, double Fx, double Fy) {
  using L = Lattice<9>;
  const double rho = P.rho0 + drho;
  const double irho = 1.0 / rho;
  const double uxd = jx * irho, uyd = jy * irho;
  const double duxd = Fx * irho, duyd = Fy * irho;  // eq. VelCorrection
  const R ux = (R)uxd, uy = (R)uyd;
  const R vx = (R)(uxd + 0.5 * duxd), vy = (R)(uyd + 0.5 * duyd);  // eq. ActualFluidVel
  const R wx = (R)(uxd + duxd), wy = (R)(uyd + duyd);
  const R uu = ux * ux + uy * uy, ww = wx * wx + wy * wy, vv = vx * vx + vy * vy;
  const R rr = (R)rho, dr = (R)drho, ph_ = (R)phi, ps_ = (R)psi;
  const R gm = (R)(3.0 * P.gphi * mphi), hm = (R)(3.0 * P.gpsi * mpsi);
  const R itf = (R)P.inv_tau, itg = (R)P.inv_tau_phi, ith = (R)P.inv_tau_psi;
  // with component densities the equilibrium carries the lattice pressure
  // c_s^2 (rho + sp): w_i sp joins every moving population, -(1 - w_0) sp
  // the rest one (zero for equal densities)
  const double spd = -(P.psh[0] * phi + P.psh[1] * psi);
  const R sp = (R)spd, drs = dr + sp;
  double gsum = 0.0, hsum = 0.0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const R w = R(L::w(i));
    const R cu = R(L::cx[i]) * ux + R(L::cy[i]) * uy;
    const R cw = R(L::cx[i]) * wx + R(L::cy[i]) * wy;
    const R pu = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    const R pw = R(3) * cw + R(4.5) * cw * cw - R(1.5) * ww;
    // f^eq(rho, u) - w_i rho0 (drho = rho - rho0)
    const R feq = i == 0 ? w * (dr + rr * pu) - R(1.0 - L::w(0)) * sp : w * (drs + rr * pu);
    const R edm = w * rr * (pw - pu);  // f^eq(rho, u + du) - f^eq(rho, u)
    pf[i] = pf[i] - (pf[i] - feq) * itf + edm;
    if (i > 0) {
      const R cv = R(L::cx[i]) * vx + R(L::cy[i]) * vy;
      const R pv = R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv;
      const R geq = w * (gm + ph_ * pv);
      const R heq = w * (hm + ps_ * pv);
      gsum += (double)geq;
      hsum += (double)heq;
      pg[i] = pg[i] - (pg[i] - geq) * itg;
      ph[i] = ph[i] - (ph[i] - heq) * ith;
    }
  }
  // rest populations close the zeroth moments (eq. EDF, i = 0)
  g0 = g0 - (g0 - (phi - gsum)) * P.inv_tau_phi;
  h0 = h0 - (h0 - (psi - hsum)) * P.inv_tau_psi;
}

// pull the populations of node (x, y), 0 <= x < nx, 0 <= y < ny, at the
// current time: population i arrives from x - c_i; across a wall it is the
// reversed population that left (x, y) (half-way bounce-back).
template <class St, typename R>
__device__ __forceinline__ void pull9(const St& src, const LBParams& P, int x, int y, R* pf, R* pg,
                                      R* ph, double& g0, double& h0) {
  using L = Lattice<9>;
  const long long here = (long long)y * P.nx + x;
  // the neighbour rows and columns, wrapped once per node
  const long long rlo = (long long)(y == 0 ? P.ny - 1 : y - 1) * P.nx;
  const long long rhi = (long long)(y == P.ny - 1 ? 0 : y + 1) * P.nx;
  const int xlo = x == 0 ? P.nx - 1 : x - 1;
  const int xhi = x == P.nx - 1 ? 0 : x + 1;
  const bool wlo = P.wall_y && y == 0;         // row y - 1 lies beyond a wall
  const bool whi = P.wall_y && y == P.ny - 1;  // row y + 1 lies beyond a wall
  pf[0] = src.template load<R>(0, 0, here);
  g0 = src.rest(1, here);
  h0 = src.rest(2, here);
#pragma unroll
  for (int i = 1; i < 9; i++) {
    const bool back = L::cy[i] > 0 ? wlo : (L::cy[i] < 0 ? whi : false);
    const long long row = L::cy[i] > 0 ? rlo : (L::cy[i] < 0 ? rhi : here - x);
    const int col = L::cx[i] > 0 ? xlo : (L::cx[i] < 0 ? xhi : x);
    const long long node = back ? here : row + col;
    const int dir = back ? L::opp[i] : i;
    pf[i] = src.template load<R>(0, dir, node);
    pg[i] = src.template load<R>(1, dir, node);
    ph[i] = src.template load<R>(2, dir, node);
  }
}

// moments of eq. MomentsDFs: the sums over the small values (f_i - w_i rho0 and
// the moving g_i, h_i) run in R, the rest populations g_0, h_0 join in FP64
template <typename R>
__device__ __forceinline__ void moments9(const R* pf, const R* pg, const R* ph, double g0, double h0,
                                         double& d, double& jx, double& jy, double& phi,
                                         double& psi) {
  using L = Lattice<9>;
  R sd = 0, sx = 0, sy = 0, sg = 0, sh = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    sd += pf[i];
    if (L::cx[i] != 0) sx += R(L::cx[i]) * pf[i];
    if (L::cy[i] != 0) sy += R(L::cy[i]) * pf[i];
    if (i > 0) {
      sg += pg[i];
      sh += ph[i];
    }
  }
  d = (double)sd;
  jx = (double)sx;
  jy = (double)sy;
  phi = g0 + (double)sg;
  psi = h0 + (double)sh;
}

// NS = 3: each iteration pulls its row and then waits for it.  NS = 4: the
// row of the next iteration is pulled at the start of this one (a register
// ring of four rows), so the loads of one row are in flight while the
// previous rows are computed.  WPE: waves per SIMD the register budget is
// sized for.
// One (strip, segment) of the lattice: the whole march of a workgroup.
// FORM 0: the force of eq. ForceFE in its potential form, -sum q grad mu_q
// over q = rho, phi, psi (eq. GradPT).  FORM 1: its divergence form,
// -div P' - psi grad kappa_c (psi - I), with the non-ideal pressure tensor P'
// of Appendix A formed per node in the U stage and its divergence taken in
// the C stage (the two forms agree up to the discretisation error).
template <class St, typename R, int BX, int NS, int FORM = 0>
__device__ __forceinline__ void lb2d_run(const St& src, const St& dst, const LBParams& P, int strip, int y0,
                                         int y1, int dir, const int* __restrict__ tflag,
                                         const int* __restrict__ tstate, const double* __restrict__ Ifield,
                                         long long* __restrict__ fib, double* __restrict__ force) {
  static_assert(NS == 3 || NS == 4, "ring of three or four rows");
  constexpr int W = BX - 4;
  __shared__ double s_m[3][3][BX];  // moment ring [slot][drho, phi, psi][lane]
  __shared__ double s_j[3][2][BX];  // momentum ring [slot][jx, jy][lane]
  // chemical-potential ring [slot][mu_rho, mu_phi, mu_psi'][lane]; with
  // FORM 1 its first field holds P'_xx instead of mu_rho
  __shared__ double s_u[3][3][BX];
  // FORM 1 only: [slot][P'_xy, P'_yy, kappa_c (psi - I)][lane]
  __shared__ double s_p[3][3][FORM == 1 ? BX : 1];

  const int j = threadIdx.x;
  const int xc = strip * W - 2 + j;
  const int x = wrap(xc, P.nx);
  const bool interior = (j >= 2) && (j < BX - 2) && (xc < P.nx);
  const int K = (y1 - y0) + 4;
  const int rbase = dir > 0 ? y0 - 2 : y1 + 1;

  const int stamp = tstate[1];  // tiles flagged with this step's stamp are active
  const int tsh = __builtin_ctz((unsigned)P.tile);  // log2 of the tile edge
  R pf[NS][9], pg[NS][9], ph[NS][9];
  double g0[NS], h0[NS];
  // tile flag of the row in each register slot, loaded with the row; the
  // membrane fields of rows k-1 and k-2 are then fetched at the start of
  // iteration k, beside the pull, instead of after a dependent flag load
  int tfl[NS];
  // NS = 4: the membrane fields a row needs (profile field on the row of the
  // chemical potential, spread force on the row of the collision) are
  // fetched one iteration early, before that iteration's stores.  Waits
  // count outstanding loads and stores in issue order, so fetched after the
  // next row's prefetch they would make the wait for them a wait for the
  // prefetch (and for the stores) as well.
  // Two register slots, alternating with the row parity (the loop is
  // unrolled by four), so no value is copied between registers while its
  // load may still be in flight.
  double Ipre_c[2] = {0.0, 0.0};
  long long fb0_c[2] = {0, 0}, fb1_c[2] = {0, 0};
  bool cact_c[2] = {false, false};

  auto load_row = [&](auto slot_c, int k) {
    constexpr int S = decltype(slot_c)::value;
    const int ry = fd_row_near(rbase + dir * k, P.ny, P.wall_y);
    pull9(src, P, x, ry, pf[S], pg[S], ph[S], g0[S], h0[S]);
    tfl[S] = tflag[(ry >> tsh) * P.ntx + (x >> tsh)];
  };

  auto body = [&](auto slot_c, int k) {
    constexpr int S = decltype(slot_c)::value;   // slot of row k
    constexpr int SN = (S + 1) % NS;             // slot of row k+1
    constexpr int SC = (S + NS - 2) % NS;        // slot of row k-2 (collided now)
    constexpr int SP = (S + NS - 1) % NS;        // slot of row k-1 (chemical potential now)
    const int r = rbase + dir * k;               // row whose moments are formed now
    if constexpr (NS == 4) {
      // unconditional (the last iteration reloads its own row), so every
      // path has the same loads in flight
      load_row(std::integral_constant<int, SN>{}, min(k + 1, K - 1));
    } else {
      load_row(std::integral_constant<int, S>{}, k);
    }
    const int qy = fd_row_near(r - dir, P.ny, P.wall_y);  // row of the chemical potential
    const int cy = r - 2 * dir;                      // row of the collision
    double Ipre = 0.0;
    long long fb0 = 0, fb1 = 0;
    bool cact;
    if constexpr (NS == 4) {
      Ipre = Ipre_c[S & 1];
      fb0 = fb0_c[S & 1];
      fb1 = fb1_c[S & 1];
      cact = cact_c[S & 1];
    } else {
      if (k >= 2 && j >= 1 && j < BX - 1 && tfl[SP] == stamp) Ipre = Ifield[(long long)qy * P.nx + x];
      cact = k >= 4 && interior && tfl[SC] == stamp;
      if (cact) {
        const long long* fp = fib + 2 * ((long long)cy * P.nx + x);
        fb0 = fp[0];
        fb1 = fp[1];
      }
    }
    // ---- M: moments of row r -> ring slot k%3
    {
      double d, jx, jy, phi, psi;
      moments9(pf[S], pg[S], ph[S], g0[S], h0[S], d, jx, jy, phi, psi);
      const int sl = k % 3;
      s_m[sl][0][j] = d;
      s_m[sl][1][j] = phi;
      s_m[sl][2][j] = psi;
      s_j[sl][0][j] = jx;
      s_j[sl][1][j] = jy;
    }
    __syncthreads();
    // ---- U: chemical potentials on the previous row -> ring slot k%3
    if (k >= 2 && j >= 1 && j < BX - 1) {
      const int a = (k + 1) % 3, b = (k + 2) % 3, c = k % 3;  // rows r-2dir, r-dir, r
      // rows a and c swap between up- and down-marching segments: each sum
      // pairs them in one addition (IEEE addition is commutative), so every
      // node gets the same rounding under any launch shape
      double lap[3], ctr[3];
#pragma unroll
      for (int f = 0; f < 3; f++) {
        const double q = s_m[b][f][j];
        const double n4 = ((s_m[b][f][j - 1] - q) + (s_m[b][f][j + 1] - q)) +
                          ((s_m[a][f][j] - q) + (s_m[c][f][j] - q));
        const double n8 = ((s_m[a][f][j - 1] - q) + (s_m[a][f][j + 1] - q)) +
                          ((s_m[c][f][j - 1] - q) + (s_m[c][f][j + 1] - q));
        // lap q = 6 sum_i w_i (q(x + c_i) - q(x)) with the D2Q9 weights
        lap[f] = (2.0 / 3.0) * n4 + (1.0 / 6.0) * n8;
        ctr[f] = q;
      }
      double mr, mp, ms;
      chem_pot(P, ctr[0], ctr[1], ctr[2], lap[0], lap[1], lap[2], Ipre, mr, mp, ms);
      const int sl = k % 3;
      if constexpr (FORM == 1) {
        // gradients of rho, phi, psi on this row (north and south resolved
        // by name, so both marching directions round alike)
        const int sn = dir > 0 ? c : a, ss = dir > 0 ? a : c;
        double gx[3], gy[3];
#pragma unroll
        for (int f = 0; f < 3; f++) {
          const double e = s_m[b][f][j + 1], wv = s_m[b][f][j - 1];
          const double nn = s_m[sn][f][j], so = s_m[ss][f][j];
          const double ne = s_m[sn][f][j + 1], nw = s_m[sn][f][j - 1];
          const double se = s_m[ss][f][j + 1], sw = s_m[ss][f][j - 1];
          gx[f] = (1.0 / 3.0) * (e - wv) + (1.0 / 12.0) * ((ne - nw) + (se - sw));
          gy[f] = (1.0 / 3.0) * (nn - so) + (1.0 / 12.0) * ((ne - se) + (nw - sw));
        }
        // P' in the concentrations C_m (eq. VariableTransform, or its form
        // with component densities), where the energy of eq. LandauFE is a
        // sum of independent terms: for each m
        // the bulk part C f_m'(C) - f_m(C) = kappa_m/2 C^2 (1-C)(1-3C) and the
        // gradient part alpha^2 kappa_m (dC dC - (|grad C|^2/2 + C lap C) I)
        double Cm[3], Xm[3], Ym[3], Lm[3];
        conc3(P, P.rho0 + ctr[0], ctr[1], ctr[2], Cm);
        conc3(P, gx[0], gx[1], gx[2], Xm);
        conc3(P, gy[0], gy[1], gy[2], Ym);
        conc3(P, lap[0], lap[1], lap[2], Lm);
        const double km[3] = {P.k1, P.k2, P.k3};
        double pb = 0.0, dd = 0.0, cl = 0.0, xy = 0.0;
#pragma unroll
        for (int m = 0; m < 3; m++) {
          const double C = Cm[m];
          pb += km[m] * (C * C * (1.0 - C) * (1.0 - 3.0 * C));
          dd += km[m] * (Xm[m] * Xm[m] - Ym[m] * Ym[m]);
          cl += km[m] * (C * Lm[m]);
          xy += km[m] * (Xm[m] * Ym[m]);
        }
        const double iso = 0.5 * pb - P.a2 * cl;
        s_u[sl][0][j] = iso + 0.5 * P.a2 * dd;
        s_p[sl][0][j] = P.a2 * xy;
        s_p[sl][1][j] = iso - 0.5 * P.a2 * dd;
        s_p[sl][2][j] = P.kc * (ctr[2] - Ipre);
      } else {
        s_u[sl][0][j] = mr;
      }
      s_u[sl][1][j] = mp;
      s_u[sl][2][j] = ms;
    }
    __syncthreads();
    if constexpr (NS == 4) {
      // the next iteration's membrane fields: its chemical-potential row is
      // row r (flag in slot S), its collision row r - dir (flag in slot SP)
      constexpr int T = SN & 1;
      const int k1 = k + 1;
      Ipre_c[T] = 0.0;
      if (k1 >= 2 && k1 < K && j >= 1 && j < BX - 1 && tfl[S] == stamp)
        Ipre_c[T] = Ifield[(long long)fd_row_near(r, P.ny, P.wall_y) * P.nx + x];
      cact_c[T] = k1 >= 4 && k1 < K && interior && tfl[SP] == stamp;
      fb0_c[T] = 0;
      fb1_c[T] = 0;
      if (cact_c[T]) {
        const long long* fp = fib + 2 * ((long long)(r - dir) * P.nx + x);
        fb0_c[T] = fp[0];
        fb1_c[T] = fp[1];
      }
    }
    // ---- C: collide row r - 2 dir with the registers of slot SC
    if (k >= 4 && interior) {
      const int a = (k + 1) % 3, b = (k + 2) % 3, c = k % 3;  // mu rows cy-dir, cy, cy+dir
      const int sn = dir > 0 ? c : a, ss = dir > 0 ? a : c;   // north (cy+1) and south (cy-1)
      // moments of row cy were stored two iterations ago (slot (k-2)%3 = a)
      const double d = s_m[a][0][j], phi = s_m[a][1][j], psi = s_m[a][2][j];
      const double jx = s_j[a][0][j], jy = s_j[a][1][j];
      double Fx, Fy;
      if constexpr (FORM == 1) {
        // -div P' - psi grad kappa_c (psi - I); the divergence of a tensor
        // column by the same stencil as a gradient, 3 sum_i w_i c_i P(x + c_i)
        double gx[4], gy[4];
        const double* fld[4][3] = {{s_u[ss][0], s_u[b][0], s_u[sn][0]},
                                   {s_p[ss][0], s_p[b][0], s_p[sn][0]},
                                   {s_p[ss][1], s_p[b][1], s_p[sn][1]},
                                   {s_p[ss][2], s_p[b][2], s_p[sn][2]}};
#pragma unroll
        for (int f = 0; f < 4; f++) {
          const double *rs = fld[f][0], *rc = fld[f][1], *rn = fld[f][2];
          const double e = rc[j + 1], wv = rc[j - 1];
          const double nn = rn[j], so = rs[j];
          const double ne = rn[j + 1], nw = rn[j - 1];
          const double se = rs[j + 1], sw = rs[j - 1];
          gx[f] = (1.0 / 3.0) * (e - wv) + (1.0 / 12.0) * ((ne - nw) + (se - sw));
          gy[f] = (1.0 / 3.0) * (nn - so) + (1.0 / 12.0) * ((ne - se) + (nw - sw));
        }
        Fx = -(gx[0] + gy[1]) - psi * gx[3];
        Fy = -(gx[1] + gy[2]) - psi * gy[3];
      } else {
        // grad mu = 3 sum_i w_i c_i mu(x + c_i)
        double gx[3], gy[3];
#pragma unroll
        for (int f = 0; f < 3; f++) {
          const double e = s_u[b][f][j + 1], wv = s_u[b][f][j - 1];
          const double nn = s_u[sn][f][j], so = s_u[ss][f][j];
          const double ne = s_u[sn][f][j + 1], nw = s_u[sn][f][j - 1];
          const double se = s_u[ss][f][j + 1], sw = s_u[ss][f][j - 1];
          gx[f] = (1.0 / 3.0) * (e - wv) + (1.0 / 12.0) * ((ne - nw) + (se - sw));
          gy[f] = (1.0 / 3.0) * (nn - so) + (1.0 / 12.0) * ((ne - se) + (nw - sw));
        }
        const double rho = P.rho0 + d;
        // thermodynamic force, eq. ForceFE with eq. GradPT (potential form)
        Fx = -(rho * gx[0] + phi * gx[1] + psi * gx[2]);
        Fy = -(rho * gy[0] + phi * gy[1] + psi * gy[2]);
      }
      Fx += P.fext[0];  // f_ext of eq. ForcingTermLBE
      Fy += P.fext[1];
      const long long node = (long long)cy * P.nx + x;
      if (cact) {
        Fx += from_fix(fb0);
        Fy += from_fix(fb1);
        fib[2 * node] = 0;
        fib[2 * node + 1] = 0;
        force[2 * node] = Fx;
        force[2 * node + 1] = Fy;
      }
      collide9(P, pf[SC], pg[SC], ph[SC], g0[SC], h0[SC], d, jx, jy, phi, psi, s_u[b][1][j],
               s_u[b][2][j], Fx, Fy);
      if constexpr (St::kQuantized) {
        // moving populations are stored rounded; the rest population of the
        // same set takes the rounding so the node's mass per set is exact
        R ef = 0, eg = 0, eh = 0;
#pragma unroll
        for (int i = 1; i < 9; i++) {
          const R qf = dst.quantize(pf[SC][i]), qg = dst.quantize(pg[SC][i]), qh = dst.quantize(ph[SC][i]);
          ef += pf[SC][i] - qf;
          eg += pg[SC][i] - qg;
          eh += ph[SC][i] - qh;
          pf[SC][i] = qf;
          pg[SC][i] = qg;
          ph[SC][i] = qh;
        }
        pf[SC][0] += ef;
        g0[SC] += (double)eg;
        h0[SC] += (double)eh;
      }
      dst.template store<R>(0, 0, node, pf[SC][0]);
      dst.store_rest(1, node, g0[SC]);
      dst.store_rest(2, node, h0[SC]);
#pragma unroll
      for (int i = 1; i < 9; i++) {
        dst.template store<R>(0, i, node, pf[SC][i]);
        dst.template store<R>(1, i, node, pg[SC][i]);
        dst.template store<R>(2, i, node, ph[SC][i]);
      }
    }
  };

  if constexpr (NS == 4) load_row(std::integral_constant<int, 0>{}, 0);
  for (int kb = 0; kb < K; kb += NS) {
    body(std::integral_constant<int, 0>{}, kb);
    if (kb + 1 < K) body(std::integral_constant<int, 1>{}, kb + 1);
    if (kb + 2 < K) body(std::integral_constant<int, 2>{}, kb + 2);
    if constexpr (NS == 4)
      if (kb + 3 < K) body(std::integral_constant<int, 3>{}, kb + 3);
  }
}

// does the (strip, rows [y0, y1)) region of a workgroup read any membrane
// field, i.e. does an active tile cover a (row, lane) whose profile field or
// spread force it reads?  (rows y0-1 .. y1 of lanes 1 .. BX-2; every thread
// of the workgroup must call it)
template <int BX>
__device__ __forceinline__ bool region_active(const LBParams& P, const int* __restrict__ tflag, int stamp,
                                              int strip, int y0, int y1) {
  const int j = threadIdx.x;
  const int x = wrap(strip * (BX - 4) - 2 + j, P.nx);
  bool a = false;
  if (j >= 1 && j < BX - 1)
    for (int r = y0 - 1; r <= y1; r++) a |= tflag[(fd_row(r, P.ny, P.wall_y) / P.tile) * P.ntx + x / P.tile] == stamp;
  return __syncthreads_or(a) != 0;
}

// The fused step over the whole lattice: one (strip, segment) per workgroup.
template <class St, typename R, int BX, int NS, int WPE, int FORM = 0>
__global__ __launch_bounds__(BX, WPE) void k_lb2d(St src, St dst, LBParams P,
                                                  const int* __restrict__ tflag,
                                                  const int* __restrict__ tstate,
                                                  const double* __restrict__ Ifield,
                                                  long long* __restrict__ fib,
                                                  double* __restrict__ force) {
  int strip, sgm;
  strip_segment((int)blockIdx.x, P.nstrip, P.nseg, P.nxcd, strip, sgm);
  const int y0 = sgm * P.seg, y1 = min(y0 + P.seg, P.ny);
  // even segments march up, odd ones down: neighbouring segments then read
  // the rows they share at the same time (both at their start or both at
  // their end)
  lb2d_run<St, R, BX, NS, FORM>(src, dst, P, strip, y0, y1, (sgm & 1) ? -1 : 1, tflag, tstate, Ifield, fib,
                                force);
}

// The same step in two passes: mode 1 takes the (strip, segment) regions
// that read no membrane field and may run beside the membrane kernels;
// mode 2 takes the others after them, each segment cut into npiece pieces of
// seg2 rows so that the few regions near the membranes still fill the GPU.
template <class St, typename R, int BX, int NS, int WPE, int FORM = 0>
__global__ __launch_bounds__(BX, WPE) void k_lb2d_part(St src, St dst, LBParams P,
                                                       const int* __restrict__ tflag,
                                                       const int* __restrict__ tstate,
                                                       const double* __restrict__ Ifield,
                                                       long long* __restrict__ fib,
                                                       double* __restrict__ force) {
  int strip, sgm, piece = 0;
  if (P.mode == 2) {
    piece = (int)blockIdx.x % P.npiece;
    const int rg = (int)blockIdx.x / P.npiece;
    strip = rg % P.nstrip;
    sgm = rg / P.nstrip;
  } else {
    strip_segment((int)blockIdx.x, P.nstrip, P.nseg, P.nxcd, strip, sgm);
  }
  int y0 = sgm * P.seg, y1 = min(y0 + P.seg, P.ny);
  if (region_active<BX>(P, tflag, tstate[1], strip, y0, y1) != (P.mode == 2)) return;
  int dir = (sgm & 1) ? -1 : 1;
  if (P.mode == 2) {
    y0 += piece * P.seg2;
    if (y0 >= y1) return;
    y1 = min(y0 + P.seg2, y1);
    dir = (piece & 1) ? -1 : 1;
  }
  lb2d_run<St, R, BX, NS, FORM>(src, dst, P, strip, y0, y1, dir, tflag, tstate, Ifield, fib, force);
}

}  // namespace lb
