// k_misc.h -- initialisation, readouts and FP64 reductions (D2Q9).
#pragma once
#include "common.h"
#include "k_ibm.h"
#include "k_lb.h"

namespace lb {

// Equilibrium populations of eq. EDF from macroscopic fields (host-staged
// doubles): rho, phi, psi, ux, uy.  mu from the Laplacians of the fields
// (mirror rows at walls) and the coupling profile.  Written in the
// post-collision convention the fused kernel pulls from: population i of
// node x lands at x - c_i, or reversed at x when that crosses a wall.
template <class St, typename R>
__global__ void k_init2d(St dst, LBParams P, const double* __restrict__ rho,
                         const double* __restrict__ phi, const double* __restrict__ psi,
                         const double* __restrict__ ux, const double* __restrict__ uy,
                         const int* __restrict__ tflag, const int* __restrict__ tstate,
                         const double* __restrict__ Ifield) {
  using L = Lattice<9>;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx), y = (int)(n / P.nx);
  const double* F[3] = {rho, phi, psi};
  double lap[3], ctr[3];
  for (int f = 0; f < 3; f++) {
    double acc = 0.0;
    ctr[f] = F[f][n];
    for (int i = 1; i < 9; i++) {
      const long long nb = (long long)fd_row(y + L::cy[i], P.ny, P.wall_y) * P.nx + wrap(x + L::cx[i], P.nx);
      acc += L::w(i) * (F[f][nb] - ctr[f]);
    }
    lap[f] = 6.0 * acc;
  }
  double I = 0;
  if (tflag[(y / P.tile) * P.ntx + x / P.tile] == tstate[1]) I = Ifield[n];
  double mr, mp, ms;
  chem_pot(P, ctr[0] - P.rho0, ctr[1], ctr[2], lap[0], lap[1], lap[2], I, mr, mp, ms);
  const double u0 = ux ? ux[n] : 0.0, u1 = uy ? uy[n] : 0.0;
  const double uu = u0 * u0 + u1 * u1;
  // lattice pressure c_s^2 (rho + sp) with component densities (sp = 0 for equal ones)
  const double sp = -(P.psh[0] * ctr[1] + P.psh[1] * ctr[2]);
  double E[3][9], gs = 0, hs = 0;
  for (int i = 0; i < 9; i++) {
    const double cu = L::cx[i] * u0 + L::cy[i] * u1;
    const double pu = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    E[0][i] = i == 0 ? L::w(0) * ((ctr[0] - P.rho0) + ctr[0] * pu) - (1.0 - L::w(0)) * sp
                     : L::w(i) * ((ctr[0] - P.rho0 + sp) + ctr[0] * pu);
    if (i > 0) {
      E[1][i] = L::w(i) * (3.0 * P.gphi * mp + ctr[1] * pu);
      E[2][i] = L::w(i) * (3.0 * P.gpsi * ms + ctr[2] * pu);
      gs += E[1][i];
      hs += E[2][i];
    }
  }
  E[1][0] = ctr[1] - gs;
  E[2][0] = ctr[2] - hs;
  if constexpr (St::kQuantized) {
    for (int s = 0; s < 3; s++)
      for (int i = 1; i < 9; i++) {
        const double q = (double)dst.quantize((R)E[s][i]);
        E[s][0] += E[s][i] - q;
        E[s][i] = q;
      }
  }
  for (int i = 0; i < 9; i++) {
    const int sy = y - L::cy[i];
    long long tn;
    int dir = i;
    if (P.wall_y && (sy < 0 || sy >= P.ny)) {
      tn = n;
      dir = L::opp[i];
    } else {
      tn = (long long)wrap(sy, P.ny) * P.nx + wrap(x - L::cx[i], P.nx);
    }
    dst.template store<R>(0, dir, tn, (R)E[0][i]);
    if (i == 0) {
      dst.store_rest(1, tn, E[1][0]);
      dst.store_rest(2, tn, E[2][0]);
    } else {
      dst.template store<R>(1, dir, tn, (R)E[1][i]);
      dst.template store<R>(2, dir, tn, (R)E[2][i]);
    }
  }
}

// moments of the current state: out = [rho, C1, C2, C3, ux, uy] x N doubles
template <class St, typename R>
__global__ void k_moments2d(St cur, LBParams P, double* __restrict__ out) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx), y = (int)(n / P.nx);
  R pf[9], pg[9], ph[9];
  double g0, h0;
  pull9(cur, P, x, y, pf, pg, ph, g0, h0);
  double d, jx, jy, phi, psi;
  moments9(pf, pg, ph, g0, h0, d, jx, jy, phi, psi);
  const double rho = P.rho0 + d;
  double C[3];
  conc3(P, rho, phi, psi, C);
  out[n] = rho;
  out[P.N + n] = C[0];
  out[2 * P.N + n] = C[1];
  out[3 * P.N + n] = C[2];
  out[4 * P.N + n] = jx / rho;
  out[5 * P.N + n] = jy / rho;
}

// per-node energy densities from the moment readout, block partial sums:
// part[blk * 8 + k] for k = mass C1..C3, F_bulk, F_grad, E_c, E_kin, p_ideal
template <int NT>
__global__ __launch_bounds__(NT) void k_energy_nodes2d(LBParams P, const double* __restrict__ mom,
                                                       const int* __restrict__ tflag,
                                                       const int* __restrict__ tstate,
                                                       const double* __restrict__ Ifield,
                                                       double* __restrict__ part) {
  using L = Lattice<9>;
  __shared__ double sh[NT / 64 + 1];
  const long long n = (long long)blockIdx.x * NT + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (n < P.N) {
    const int x = (int)(n % P.nx), y = (int)(n / P.nx);
    const double kap[3] = {P.k1, P.k2, P.k3};
    for (int m = 0; m < 3; m++) {
      const double* C = mom + (long long)(1 + m) * P.N;
      const double c = C[n];
      double gx = 0, gy = 0;
      for (int i = 1; i < 9; i++) {
        const long long nb = (long long)fd_row(y + L::cy[i], P.ny, P.wall_y) * P.nx + wrap(x + L::cx[i], P.nx);
        gx += L::w(i) * L::cx[i] * C[nb];
        gy += L::w(i) * L::cy[i] * C[nb];
      }
      gx *= 3.0;
      gy *= 3.0;
      v[m] = c;
      v[3] += 0.5 * kap[m] * c * c * (1.0 - c) * (1.0 - c);
      v[4] += 0.5 * P.a2 * kap[m] * (gx * gx + gy * gy);
    }
    double I = 0;
    if (tflag[(y / P.tile) * P.ntx + x / P.tile] == tstate[1]) I = Ifield[n];
    const double psi = mom[3 * P.N + n];
    v[5] = 0.5 * P.kc * (psi - I) * (psi - I);
    const double rho = mom[n], ux = mom[4 * P.N + n], uy = mom[5 * P.N + n];
    v[6] = 0.5 * rho * (ux * ux + uy * uy);
    // c_s^2 rho ln rho; with component densities the ideal gas is that of
    // the number density n = sum_m C_m, c_s^2 M_b n ln n
    if (P.dens) {
      const double nn = mom[P.N + n] + mom[2 * P.N + n] + mom[3 * P.N + n];
      v[7] = P.mb * nn * log(nn) / 3.0;
    } else {
      v[7] = rho * log(rho) / 3.0;
    }
  }
  for (int k = 0; k < 8; k++) {
    const double s = block_sum<NT>(v[k], sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * 8 + k] = s;
  }
}

// per-marker strain (segment l) and bending (vertex l) energies of a ring
__global__ void k_memenergy2d(MemDev md, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= md.M) return;
  const int m = md.mid[g];
  const int b = md.moff[m], n = md.moff[m + 1] - b;
  const int l = g - b;
  const int lp = b + (l + 1) % n, lm = b + (l + n - 1) % n;
  const double ex = md.X[3 * lp] - md.X[3 * g], ey = md.X[3 * lp + 1] - md.X[3 * g + 1];
  const double len = sqrt(ex * ex + ey * ey);
  out[2 * g] = seg_energy(md.law[m], md.ks[m], len / md.rest[g]) * md.rest[g];
  double gax, gay, gbx, gby, e;
  bend_grad(ex, ey, md.X[3 * g] - md.X[3 * lm], md.X[3 * g + 1] - md.X[3 * lm + 1], md.kb[m], gax, gay,
            gbx, gby, e);
  out[2 * g + 1] = e;
}

// sum of nrows rows of width w (row-major) in fixed order -> out[w]
template <int NT>
__global__ __launch_bounds__(NT) void k_sum_rows(const double* __restrict__ in, long long nrows,
                                                 int w, double* __restrict__ out) {
  __shared__ double sh[NT / 64 + 1];
  for (int k = 0; k < w; k++) {
    double acc = 0;
    for (long long r = threadIdx.x; r < nrows; r += NT) acc += in[r * w + k];
    const double s = block_sum<NT>(acc, sh);
    if (threadIdx.x == 0) out[k] = s;
  }
}

// largest |population| and a count of non-finite entries (failure detection)
template <class St, typename R, int NT>
__global__ __launch_bounds__(NT) void k_check(St cur, long long N, int Q, int* __restrict__ bad) {
  const long long n = (long long)blockIdx.x * NT + threadIdx.x;
  if (n >= N) return;
  for (int s = 0; s < 3; s++)
    for (int i = 0; i < Q; i++) {
      const double v = cur.template load<double>(s, i, n);
      if (!isfinite(v)) atomicOr(bad, 1);
    }
}

}  // namespace lb
