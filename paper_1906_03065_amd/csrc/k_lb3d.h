// k_lb3d.h -- the lattice-Boltzmann step (Sec. 3.1) on D3Q19.
//
// Two kernels per step:
//   k_mom3d   pull-streams every node and writes its moments drho, phi and
//             psi (FP64) to a moment field (24 B per node);
//   k_lb3d    a workgroup of 256 threads owns a TX x TY column of nodes
//             (TX TY = 256; 16 x 16, 32 x 8 or 64 x 4) and marches along z.
//             Per plane it stages the moments of the (TX+4) x (TY+4) region
//             in an LDS ring, forms mu on the inner (TX+2) x (TY+2) region
//             (Appendix A), then for its TX x TY nodes pulls the populations,
//             forms grad mu,
//             the force (eqs. ForcingTermLBE, ForceFE + the spread membrane
//             force) and collides (eq. LBE).
// In 3D the two-node halo of the mu chain would make a single-pass kernel
// re-read the 55 populations of (T+4)^2/T^2 as many nodes; staging 24 B of
// moments instead costs one extra read of the populations per step.
// Precision follows the 2D kernel: moments, mu and grad mu in FP64.
#pragma once
#include "common.h"
#include "k_lb.h"
#include "store.h"

namespace lb {

constexpr int T3 = 32;  // default tile extent in x (y: 256 / T3)

struct Moments3 {
  double* d;     // drho = rho - 1
  double* phi;
  double* psi;
};

// pull the populations of node (x, y, z), each index within the lattice;
// bounce-back across walls in y, z
template <class St, typename R>
__device__ __forceinline__ void pull19(const St& src, const LBParams& P, int x, int y, int z, R* pf,
                                       R* pg, R* ph, double& g0, double& h0) {
  using L = Lattice<19>;
  const long long plane = (long long)P.ny * P.nx;
  const long long zc = z * plane;
  const long long here = zc + (long long)y * P.nx + x;
  // the neighbour planes, rows and columns, wrapped once per node
  const long long zlo = (z == 0 ? P.nz - 1 : z - 1) * plane, zhi = (z == P.nz - 1 ? 0 : z + 1) * plane;
  const long long ylo = (long long)(y == 0 ? P.ny - 1 : y - 1) * P.nx;
  const long long yhi = (long long)(y == P.ny - 1 ? 0 : y + 1) * P.nx, yc = (long long)y * P.nx;
  const int xlo = x == 0 ? P.nx - 1 : x - 1;
  const int xhi = x == P.nx - 1 ? 0 : x + 1;
  const bool wylo = P.wall_y && y == 0, wyhi = P.wall_y && y == P.ny - 1;  // beyond a wall in y
  const bool wzlo = P.wall_z && z == 0, wzhi = P.wall_z && z == P.nz - 1;  // beyond a wall in z
  pf[0] = src.template load<R>(0, 0, here);
  g0 = src.rest(1, here);
  h0 = src.rest(2, here);
#pragma unroll
  for (int i = 1; i < 19; i++) {
    const bool back = (L::cy[i] > 0 ? wylo : (L::cy[i] < 0 ? wyhi : false)) ||
                      (L::cz[i] > 0 ? wzlo : (L::cz[i] < 0 ? wzhi : false));
    const long long zo = L::cz[i] > 0 ? zlo : (L::cz[i] < 0 ? zhi : zc);
    const long long yo = L::cy[i] > 0 ? ylo : (L::cy[i] < 0 ? yhi : yc);
    const int xo = L::cx[i] > 0 ? xlo : (L::cx[i] < 0 ? xhi : x);
    const long long node = back ? here : zo + yo + xo;
    const int dir = back ? L::opp[i] : i;
    pf[i] = src.template load<R>(0, dir, node);
    pg[i] = src.template load<R>(1, dir, node);
    ph[i] = src.template load<R>(2, dir, node);
  }
}

template <typename R>
__device__ __forceinline__ void moments19(const R* pf, const R* pg, const R* ph, double g0, double h0,
                                          double& d, double& jx, double& jy, double& jz, double& phi,
                                          double& psi) {
  using L = Lattice<19>;
  R sd = 0, sx = 0, sy = 0, sz = 0, sg = 0, sh = 0;
#pragma unroll
  for (int i = 0; i < 19; i++) {
    sd += pf[i];
    if (L::cx[i] != 0) sx += R(L::cx[i]) * pf[i];
    if (L::cy[i] != 0) sy += R(L::cy[i]) * pf[i];
    if (L::cz[i] != 0) sz += R(L::cz[i]) * pf[i];
    if (i > 0) {
      sg += pg[i];
      sh += ph[i];
    }
  }
  d = (double)sd;
  jx = (double)sx;
  jy = (double)sy;
  jz = (double)sz;
  phi = g0 + (double)sg;
  psi = h0 + (double)sh;
}

template <class St, typename R>
__global__ __launch_bounds__(256) void k_mom3d(St src, LBParams P, Moments3 M) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
  R pf[19], pg[19], ph[19];
  double g0, h0, d, jx, jy, jz, phi, psi;
  pull19(src, P, x, y, z, pf, pg, ph, g0, h0);
  moments19(pf, pg, ph, g0, h0, d, jx, jy, jz, phi, psi);
  M.d[n] = d;
  M.phi[n] = phi;
  M.psi[n] = psi;
}

// BGK + exact-difference collision of one D3Q19 node, in place
template <typename R>
__device__ __forceinline__ void collide19(const LBParams& P, R* pf, R* pg, R* ph, double& g0,
                                          double& h0, double drho, double jx, double jy, double jz,
                                          double phi, double psi, double mphi, double mpsi,
                                          double Fx, double Fy, double Fz) {
  using L = Lattice<19>;
  const double rho = P.rho0 + drho;
  const double irho = 1.0 / rho;
  const double uxd = jx * irho, uyd = jy * irho, uzd = jz * irho;
  const double dxd = Fx * irho, dyd = Fy * irho, dzd = Fz * irho;  // eq. VelCorrection
  const R ux = (R)uxd, uy = (R)uyd, uz = (R)uzd;
  const R vx = (R)(uxd + 0.5 * dxd), vy = (R)(uyd + 0.5 * dyd), vz = (R)(uzd + 0.5 * dzd);
  const R wx = (R)(uxd + dxd), wy = (R)(uyd + dyd), wz = (R)(uzd + dzd);
  const R uu = ux * ux + uy * uy + uz * uz, ww = wx * wx + wy * wy + wz * wz;
  const R vv = vx * vx + vy * vy + vz * vz;
  const R rr = (R)rho, dr = (R)drho, ph_ = (R)phi, ps_ = (R)psi;
  const R gm = (R)(3.0 * P.gphi * mphi), hm = (R)(3.0 * P.gpsi * mpsi);
  const R itf = (R)P.inv_tau, itg = (R)P.inv_tau_phi, ith = (R)P.inv_tau_psi;
  // lattice pressure c_s^2 (rho + sp) with component densities (sp = 0 for equal ones)
  const double spd = -(P.psh[0] * phi + P.psh[1] * psi);
  const R sp = (R)spd, drs = dr + sp;
  double gsum = 0.0, hsum = 0.0;
#pragma unroll
  for (int i = 0; i < 19; i++) {
    const R w = R(L::w(i));
    const R cu = R(L::cx[i]) * ux + R(L::cy[i]) * uy + R(L::cz[i]) * uz;
    const R cw = R(L::cx[i]) * wx + R(L::cy[i]) * wy + R(L::cz[i]) * wz;
    const R pu = R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu;
    const R pw = R(3) * cw + R(4.5) * cw * cw - R(1.5) * ww;
    const R feq = i == 0 ? w * (dr + rr * pu) - R(1.0 - L::w(0)) * sp : w * (drs + rr * pu);
    const R edm = w * rr * (pw - pu);
    pf[i] = pf[i] - (pf[i] - feq) * itf + edm;
    if (i > 0) {
      const R cv = R(L::cx[i]) * vx + R(L::cy[i]) * vy + R(L::cz[i]) * vz;
      const R pv = R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv;
      const R geq = w * (gm + ph_ * pv);
      const R heq = w * (hm + ps_ * pv);
      gsum += (double)geq;
      hsum += (double)heq;
      pg[i] = pg[i] - (pg[i] - geq) * itg;
      ph[i] = ph[i] - (ph[i] - heq) * ith;
    }
  }
  g0 = g0 - (g0 - (phi - gsum)) * P.inv_tau_phi;
  h0 = h0 - (h0 - (psi - hsum)) * P.inv_tau_psi;
}

// row of a staged halo node: rows beyond the two-node ghost band of a wall
// are never used (they only occur in a ragged last tile of a lattice thinner
// than the tile), so they are clamped into the band to stay in bounds
__device__ __forceinline__ int halo_row(int v, int n, int wall) {
  if (wall) v = min(max(v, -2), n + 1);
  return fd_row(v, n, wall);
}

__device__ __forceinline__ int tile3(const LBParams& P, int x, int y, int z) {
  return ((z / P.tile) * P.nty + y / P.tile) * P.ntx + x / P.tile;
}

// TX: tile extent in x (wider tiles read whole cache lines of each x row)
template <class St, typename R, int TX = T3>
__global__ __launch_bounds__(256, 2) void k_lb3d(St src, St dst, LBParams P, Moments3 M,
                                                 const int* __restrict__ tflag,
                                                 const int* __restrict__ tstate,
                                                 const double* __restrict__ Ifield,
                                                 long long* __restrict__ fib,
                                                 double* __restrict__ force, int ntilex) {
  using L = Lattice<19>;
  static_assert(TX == 16 || TX == 32 || TX == 64, "tile of 256 nodes");
  constexpr int TY = 256 / TX;
  constexpr int TXH = TX + 4, TYH = TY + 4;  // with the two-node halo
  constexpr int TXU = TX + 2, TYU = TY + 2;  // region where mu is formed
  constexpr int NH = (TXH * TYH + 255) / 256, NU = (TXU * TYU + 255) / 256;  // passes of 256 threads
  __shared__ double s_m[3][3][TXH * TYH];  // moments ring: drho, phi, psi
  __shared__ double s_u[3][3][TXU * TYU];  // chemical-potential ring
  const int tid = threadIdx.x;
  // (tile, segment) of this workgroup: each XCD gets a contiguous run of
  // the tile order, so tiles that share halo lines meet in one L2
  int tl, sgm;
  strip_segment((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)gridDim.x, (int)gridDim.y, P.nxcd, tl, sgm);
  const int tx = tl % ntilex, ty = tl / ntilex;
  const int x0 = tx * TX, y0t = ty * TY;
  const int z0 = sgm * P.seg;
  const int z1 = min(z0 + P.seg, P.nz);
  const int K = (z1 - z0) + 4;
  const int dir = (sgm & 1) ? -1 : 1;
  const int zbase = dir > 0 ? z0 - 2 : z1 + 1;
  const int stamp = tstate[1];
  // this thread's interior node
  const int ix = tid % TX, iy = tid / TX;
  const int gx = x0 + ix, gy = y0t + iy;
  const bool own = gx < P.nx && gy < P.ny;
  const int xw = wrap(gx, P.nx);

  // tile flags of this thread's chemical-potential nodes and collision node,
  // loaded one plane ahead so that every load of an iteration (moments,
  // profile field, pull, spread force) is issued before the first wait
  int fU[NU] = {}, fC = 0;
  // the populations of plane z_j are pulled at iteration j + 1 into register
  // set j & 1 and collided at iteration j + 2: the next plane's pull is in
  // flight while the current one is computed
  R pf[2][19], pg[2][19], ph[2][19];
  double g0[2] = {0.0, 0.0}, h0[2] = {0.0, 0.0};
  auto body = [&](auto set_c, int k) {
    constexpr int S = decltype(set_c)::value;  // set collided now (k & 1)
    constexpr int SN = S ^ 1;                  // set pulled now
    const int zk = zbase + dir * k;
    const int slot = k % 3;
    // Loads are issued with the ones under a condition first and the
    // unconditional ones in the order they are consumed: waits count
    // outstanding loads and stores in issue order, so a conditional load
    // issued after another would leave the wait for the earlier one unsure
    // of its count, and it would then wait for everything (the next plane's
    // pull included).
    // ---- issue: the spread force of plane z_{k-2} (collided now)
    const int cz = zk - 2 * dir;
    const bool doC = k >= 4 && own;
    const bool cact = doC && fC == stamp;
    const long long node = ((long long)cz * P.ny + gy) * P.nx + xw;
    long long fb[3] = {0, 0, 0};
    if (cact)
      for (int a3 = 0; a3 < 3; a3++) fb[a3] = fib[3 * node + a3];
    // ---- issue: profile field of plane z_{k-1} where its tile is active,
    // tile flags of the next plane's chemical-potential nodes
    const int zr = halo_row(zk, P.nz, P.wall_z);
    const int zq = halo_row(zk - dir, P.nz, P.wall_z);
    double Iv[NU] = {};
    int nfU[NU] = {};
#pragma unroll
    for (int r = 0; r < NU; r++) {
      const int q = tid + 256 * r;
      if (q < TXU * TYU) {
        const int xx = wrap(x0 - 1 + q % TXU, P.nx);
        const int yy = halo_row(y0t - 1 + q / TXU, P.ny, P.wall_y);
        if (k + 1 < K) nfU[r] = tflag[tile3(P, xx, yy, zr)];
        if (k >= 2 && fU[r] == stamp) Iv[r] = Ifield[((long long)zq * P.ny + yy) * P.nx + xx];
      }
    }
    // ---- issue: tile flag of the next collision node (consumed at the
    // start of the next iteration, so issued before the bulk of this one's loads)
    const int pz = min(max(zk - dir, 0), P.nz - 1), gyc = min(gy, P.ny - 1);
    const int nfC = tflag[tile3(P, xw, gyc, pz)];
    // ---- issue: moments of plane zk on the (TX+4) x (TY+4) region (lanes
    // past the region load its last node again, unused)
    double mv[NH][3];
#pragma unroll
    for (int r = 0; r < NH; r++) {
      const int q = min(tid + 256 * r, TXH * TYH - 1);
      const int hx = q % TXH, hy = q / TXH;
      const int xx = wrap(x0 - 2 + hx, P.nx);
      const int yy = halo_row(y0t - 2 + hy, P.ny, P.wall_y);
      const long long nd = ((long long)zr * P.ny + yy) * P.nx + xx;
      mv[r][0] = M.d[nd];
      mv[r][1] = M.phi[nd];
      mv[r][2] = M.psi[nd];
    }
    // ---- issue: pull of plane z_{k-1} (collided next iteration), on every
    // iteration and lane (a plane or row outside the lattice is clamped into
    // it; only the pulls of iterations 3 .. K-2 at the workgroup's own nodes
    // are collided)
    pull19(src, P, xw, gyc, pz, pf[SN], pg[SN], ph[SN], g0[SN], h0[SN]);
    // ---- L: moments to the ring
#pragma unroll
    for (int r = 0; r < NH; r++) {
      const int q = tid + 256 * r;
      if (q < TXH * TYH) {
        s_m[slot][0][q] = mv[r][0];
        s_m[slot][1][q] = mv[r][1];
        s_m[slot][2][q] = mv[r][2];
      }
    }
    __syncthreads();
    // ---- U: mu on plane z_{k-1} over the (TX+2) x (TY+2) region
    if (k >= 2) {
      const int a = (k + 1) % 3, b = (k + 2) % 3, c = slot;  // planes z_{k-2}, z_{k-1}, z_k
      const int pa = dir > 0 ? a : c, pc = dir > 0 ? c : a;   // planes below / above in z
#pragma unroll
      for (int r = 0; r < NU; r++) {
        const int q = tid + 256 * r;
        if (q >= TXU * TYU) continue;
        const int ux_ = q % TXU, uy_ = q / TXU;
        const int hq = (uy_ + 1) * TXH + (ux_ + 1);  // centre in the staged region
        double lap[3], ctr[3];
#pragma unroll
        for (int f = 0; f < 3; f++) {
          const double qc = s_m[b][f][hq];
          double acc = 0.0;
#pragma unroll
          for (int i = 1; i < 19; i++) {
            const int pl = L::cz[i] > 0 ? pc : (L::cz[i] < 0 ? pa : b);
            acc += L::w(i) * (s_m[pl][f][hq + L::cy[i] * TXH + L::cx[i]] - qc);
          }
          lap[f] = 6.0 * acc;
          ctr[f] = qc;
        }
        double mr, mp, ms;
        chem_pot(P, ctr[0], ctr[1], ctr[2], lap[0], lap[1], lap[2], Iv[r], mr, mp, ms);
        s_u[slot][0][q] = mr;
        s_u[slot][1][q] = mp;
        s_u[slot][2][q] = ms;
      }
    }
    __syncthreads();
    // ---- C: collide plane z_{k-2}
    if (doC) {
      const int a = (k + 1) % 3, b = (k + 2) % 3, c = slot;  // mu planes z_{k-3}, z_{k-2}, z_{k-1}
      const int pa = dir > 0 ? a : c, pc = dir > 0 ? c : a;
      R* pfc = pf[S];
      R* pgc = pg[S];
      R* phc = ph[S];
      double& g0c = g0[S];
      double& h0c = h0[S];
      double d, jx, jy, jz, phi, psi;
      moments19(pfc, pgc, phc, g0c, h0c, d, jx, jy, jz, phi, psi);
      const int uq = (iy + 1) * TXU + (ix + 1);
      double gr[3][3];
#pragma unroll
      for (int f = 0; f < 3; f++) {
        double sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int i = 1; i < 19; i++) {
          const int pl = L::cz[i] > 0 ? pc : (L::cz[i] < 0 ? pa : b);
          const double v = L::w(i) * s_u[pl][f][uq + L::cy[i] * TXU + L::cx[i]];
          sx += L::cx[i] * v;
          sy += L::cy[i] * v;
          sz += L::cz[i] * v;
        }
        gr[f][0] = 3.0 * sx;
        gr[f][1] = 3.0 * sy;
        gr[f][2] = 3.0 * sz;
      }
      const double rho = P.rho0 + d;
      double F[3];
      for (int a3 = 0; a3 < 3; a3++)  // plus f_ext of eq. ForcingTermLBE
        F[a3] = -(rho * gr[0][a3] + phi * gr[1][a3] + psi * gr[2][a3]) + P.fext[a3];
      if (cact) {
        for (int a3 = 0; a3 < 3; a3++) {
          // keeps the conversion (and so the wait for the load) here rather
          // than next to the load, where waiting would include every later load
          asm volatile("" : "+v"(fb[a3]));
          F[a3] += from_fix(fb[a3]);
          fib[3 * node + a3] = 0;
          force[3 * node + a3] = F[a3];
        }
      }
      collide19(P, pfc, pgc, phc, g0c, h0c, d, jx, jy, jz, phi, psi, s_u[b][1][uq], s_u[b][2][uq], F[0], F[1],
                F[2]);
      if constexpr (St::kQuantized) {
        R ef = 0, eg = 0, eh = 0;
#pragma unroll
        for (int i = 1; i < 19; i++) {
          const R qf = dst.quantize(pfc[i]), qg = dst.quantize(pgc[i]), qh = dst.quantize(phc[i]);
          ef += pfc[i] - qf;
          eg += pgc[i] - qg;
          eh += phc[i] - qh;
          pfc[i] = qf;
          pgc[i] = qg;
          phc[i] = qh;
        }
        pfc[0] += ef;
        g0c += (double)eg;
        h0c += (double)eh;
      }
      dst.template store<R>(0, 0, node, pfc[0]);
      dst.store_rest(1, node, g0c);
      dst.store_rest(2, node, h0c);
#pragma unroll
      for (int i = 1; i < 19; i++) {
        dst.template store<R>(0, i, node, pfc[i]);
        dst.template store<R>(1, i, node, pgc[i]);
        dst.template store<R>(2, i, node, phc[i]);
      }
    }
#pragma unroll
    for (int r = 0; r < NU; r++) fU[r] = nfU[r];
    fC = nfC;
    __syncthreads();  // the rings are rewritten by the next plane
  };
  for (int k = 0; k < K; k += 2) {
    body(std::integral_constant<int, 0>{}, k);
    if (k + 1 < K) body(std::integral_constant<int, 1>{}, k + 1);
  }
}

}  // namespace lb
