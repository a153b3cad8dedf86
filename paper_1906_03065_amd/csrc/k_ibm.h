// k_ibm.h -- membrane side of the step for 2D ring membranes: active-tile
// map, coupling profile I and coupling force (Sec. 2.4 eq. Iprofile, Sec. 3.2
// eqs. DiscreteCE/DiscreteCF), strain and bending forces (eqs. DiscreteSF,
// DiscreteBF), spreading (eq. Spreading) and interpolation + Euler update
// (eqs. Interpolation, UpdatedXl).  All marker arithmetic is FP64.
//
// Active tiles: every lattice tile (TILE x TILE nodes) that meets a
// membrane's bounding box grown by r_cut + 3.  Only these tiles carry a
// profile I different from 0, a spread force, or a stored total force; the
// fused lattice kernel reads the maps there and nowhere else.
//
// Signed distance d(x): distance to the closest segment of the marker
// polygon, positive inside.  Inside/outside is the even-odd rule: the parity
// of the tile centre from a ray towards +x over all segments, then flipped
// once per segment crossing the short path from the tile centre to the node
// (such segments lie within reach of the tile and are among its candidates).
#pragma once
#include "common.h"
#include "k_lb.h"

namespace lb {

constexpr int TILE2 = 16;         // 2D tile edge
constexpr int COUP_THREADS = 256; // one thread per node of a 16x16 tile

struct MemDev {
  double* X;          // 3 per marker
  double* U;          // 3 per marker
  double* F;          // 3 per marker, total force of the last step
  long long* Facc;    // 3 per marker, fixed-point coupling force accumulator
  double* rest;       // rest length of segment l -> l+1 (2D)
  int* moff;          // K+1 offsets
  int* mid;           // membrane id of every marker
  double* ks;         // K
  double* kb;         // K
  double* mbox;       // 6 per membrane: lo xyz, hi xyz
  int* status;        // [0] fixed-point overflow, [1] lattice too small for a membrane
  int K, M;
};

struct TileMap {
  int* tflag;         // per tile: 1 active
  int* tlist;         // active tiles
  int* tcount;        // number of active tiles
  int ntx, nty, ntz, tile;
};

// ---------------------------------------------------------------------------
// block-wide reductions (fixed order: wave shuffles then a serial pass over
// the waves), used where results must be bitwise reproducible
template <int NT>
__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; i++) t += sh[i];
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  t = sh[0];
  __syncthreads();
  return t;
}

template <int NT>
__device__ int block_sum_int(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  int t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; i++) t += sh[i];
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = t;
  __syncthreads();
  t = sh[0];
  __syncthreads();
  return t;
}

template <int NT>
__device__ double block_min(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 1; i < NT / 64; i++) sh[0] = fmin(sh[0], sh[i]);
  __syncthreads();
  double t = sh[0];
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// bounding boxes and the active-tile map; one workgroup per simulation
template <int NT>
__global__ __launch_bounds__(NT) void k_tiles(MemDev md, TileMap tm, int nx, int ny, int nz,
                                              int wall_y, int wall_z, int D, double reach) {
  __shared__ double sh[NT / 64 + 1];
  __shared__ int cnt;
  const int tid = threadIdx.x;
  // clear the previous map
  const int nprev = *tm.tcount;
  for (int i = tid; i < nprev; i += NT) tm.tflag[tm.tlist[i]] = 0;
  if (tid == 0) cnt = 0;
  __syncthreads();
  for (int m = 0; m < md.K; m++) {
    const int b = md.moff[m], e = md.moff[m + 1];
    double lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
      double mn = 1e300, mx = -1e300;
      if (a < D)
        for (int l = b + tid; l < e; l += NT) {
          const double v = md.X[3 * l + a];
          mn = fmin(mn, v);
          mx = fmax(mx, v);
        }
      lo[a] = block_min<NT>(mn, sh);
      hi[a] = -block_min<NT>(-mx, sh);
    }
    if (tid == 0)
      for (int a = 0; a < 3; a++) {
        md.mbox[6 * m + a] = lo[a];
        md.mbox[6 * m + 3 + a] = hi[a];
      }
    // non-finite or runaway markers: flag and leave this membrane off the map
    bool sane = true;
    for (int a = 0; a < D; a++)
      if (!(fabs(lo[a]) < 1e9) || !(fabs(hi[a]) < 1e9)) sane = false;
    if (!sane) {
      if (tid == 0) md.status[0] = 1;
      __syncthreads();
      continue;
    }
    // the periodic image of a node must be unique within the grown box
    const int dims[3] = {nx, ny, nz};
    const int per[3] = {1, !wall_y, !wall_z};
    for (int a = 0; a < D; a++)
      if (per[a] && hi[a] - lo[a] + 2.0 * reach + 2.0 * tm.tile >= dims[a] && tid == 0)
        md.status[1] = 1;
    // tile ranges of the grown box
    int t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0}, nt[3] = {tm.ntx, tm.nty, tm.ntz};
    for (int a = 0; a < D; a++) {
      t0[a] = (int)floor((lo[a] - reach) / tm.tile);
      t1[a] = (int)floor((hi[a] + reach) / tm.tile);
      if (!per[a]) {
        t0[a] = max(t0[a], 0);
        t1[a] = min(t1[a], nt[a] - 1);
      } else if (t1[a] - t0[a] + 1 > nt[a]) {
        t0[a] = 0;
        t1[a] = nt[a] - 1;
      }
    }
    const int sx = t1[0] - t0[0] + 1, sy = t1[1] - t0[1] + 1, sz = (D == 3) ? t1[2] - t0[2] + 1 : 1;
    const long long total = (long long)sx * sy * sz;
    for (long long q = tid; q < total; q += NT) {
      const int ix = (int)(q % sx), iy = (int)((q / sx) % sy), iz = (int)(q / ((long long)sx * sy));
      const int tx = wrap(t0[0] + ix, nt[0]), ty = wrap(t0[1] + iy, nt[1]);
      const int tz = (D == 3) ? wrap(t0[2] + iz, nt[2]) : 0;
      const int t = (tz * tm.nty + ty) * tm.ntx + tx;
      if (atomicCAS(&tm.tflag[t], 0, 1) == 0) tm.tlist[atomicAdd(&cnt, 1)] = t;
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) *tm.tcount = cnt;
}

// ---------------------------------------------------------------------------
// 2D geometry helpers (FP64)

// closest point of segment A-B to P: squared distance and parameter t
__device__ __forceinline__ double seg_d2(double px, double py, double ax, double ay, double bx,
                                         double by, double& t) {
  const double ex = bx - ax, ey = by - ay;
  const double qx = px - ax, qy = py - ay;
  const double ee = ex * ex + ey * ey;
  double s = ee > 0.0 ? (qx * ex + qy * ey) / ee : 0.0;
  s = fmin(fmax(s, 0.0), 1.0);
  const double dx = qx - s * ex, dy = qy - s * ey;
  t = s;
  return dx * dx + dy * dy;
}

// does the ray from P towards +x cross segment A-B (half-open in y)?
__device__ __forceinline__ int ray_cross(double px, double py, double ax, double ay, double bx,
                                         double by) {
  if ((ay > py) != (by > py)) {
    const double xc = ax + (py - ay) * (bx - ax) / (by - ay);
    return px < xc;
  }
  return 0;
}

__device__ __forceinline__ double orient(double ax, double ay, double bx, double by, double cx,
                                         double cy) {
  return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// does the path P->Q cross segment A-B?  Half-open on both (a vertex on the
// path is counted by exactly one of its two segments)
__device__ __forceinline__ int path_cross(double px, double py, double qx, double qy, double ax,
                                          double ay, double bx, double by) {
  const double o1 = orient(px, py, qx, qy, ax, ay), o2 = orient(px, py, qx, qy, bx, by);
  if ((o1 >= 0.0) == (o2 >= 0.0)) return 0;
  const double o3 = orient(ax, ay, bx, by, px, py), o4 = orient(ax, ay, bx, by, qx, qy);
  return (o3 >= 0.0) != (o4 >= 0.0);
}

__device__ __forceinline__ double near_image(double v, double c, int n) {
  return v + n * floor((c - v) / n + 0.5);
}

struct CoupArgs {
  int nx, ny, wall_y;
  double alpha, kappa_c, r_cut;
  int want_force;
};

// per node: signed distance to membrane m, closest segment and its t; the
// caller's block cooperates on candidate culling.  Returns via refs; d2 =
// +inf when the node lies outside the membrane's grown box.
template <int NT>
__device__ void ring_geometry(const MemDev& md, const CoupArgs& ca, int m, double px_tile,
                              double py_tile, double px, double py, bool valid_node, double& d2_best,
                              int& seg_best, double& t_best, int& inside, int* s_cand, int* s_int,
                              double* s_dbl) {
  const int b = md.moff[m], n = md.moff[m + 1] - b;
  const double* X = md.X + 3 * b;
  const double reach = ca.r_cut + 1.0;
  const double hd = 0.5 * TILE2 * 1.41421356237309515 + 1e-9;
  const double cull = ca.r_cut + hd + 1.0;
  // parity of the tile centre: ray towards +x over all segments
  int cr = 0;
  for (int l = threadIdx.x; l < n; l += NT) {
    const int l1 = (l + 1 == n) ? 0 : l + 1;
    cr += ray_cross(px_tile, py_tile, X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1]);
  }
  const int parity = block_sum_int<NT>(cr, s_int) & 1;
  d2_best = 1e300;
  seg_best = -1;
  t_best = 0.0;
  int flips = 0;
  for (int c0 = 0; c0 < n; c0 += NT) {
    if (threadIdx.x == 0) s_int[NT / 64] = 0;
    __syncthreads();
    const int l = c0 + threadIdx.x;
    if (l < n) {
      const int l1 = (l + 1 == n) ? 0 : l + 1;
      double t;
      const double d2 = seg_d2(px_tile, py_tile, X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1], t);
      if (d2 <= cull * cull) s_cand[atomicAdd(&s_int[NT / 64], 1)] = l;
    }
    __syncthreads();
    const int nc = s_int[NT / 64];
    if (valid_node)
      for (int q = 0; q < nc; q++) {
        const int s = s_cand[q];
        const int s1 = (s + 1 == n) ? 0 : s + 1;
        const double ax = X[3 * s], ay = X[3 * s + 1], bx = X[3 * s1], by = X[3 * s1 + 1];
        double t;
        const double d2 = seg_d2(px, py, ax, ay, bx, by, t);
        if (d2 < d2_best || (d2 == d2_best && s < seg_best)) {
          d2_best = d2;
          seg_best = s;
          t_best = t;
        }
        flips += path_cross(px_tile, py_tile, px, py, ax, ay, bx, by);
      }
    __syncthreads();
  }
  inside = parity ^ (flips & 1);
  (void)reach;
  (void)s_dbl;
}

template <class St, typename R, int NT>
__global__ __launch_bounds__(NT) void k_coupling2d(MemDev md, TileMap tm, CoupArgs ca,
                                                   double* __restrict__ Ifield, St cur) {
  __shared__ int s_cand[NT];
  __shared__ int s_int[NT / 64 + 2];
  __shared__ double s_dbl[NT / 64 + 1];
  const int ntl = *tm.tcount;
  const double reach = ca.r_cut + 1.0;
  for (int li = blockIdx.x; li < ntl; li += gridDim.x) {
    const int t = tm.tlist[li];
    const int tx = t % tm.ntx, ty = t / tm.ntx;
    const int x = tx * TILE2 + (threadIdx.x % TILE2), y = ty * TILE2 + (threadIdx.x / TILE2);
    const bool valid = (x < ca.nx) && (y < ca.ny);
    const double xt = tx * TILE2 + 0.5 * (TILE2 - 1), yt = ty * TILE2 + 0.5 * (TILE2 - 1);
    double Itot = 0.0;
    // pass 1: the profile, summed over membranes
    for (int m = 0; m < md.K; m++) {
      const double* bx = md.mbox + 6 * m;
      const double cx = 0.5 * (bx[0] + bx[3]), cy = 0.5 * (bx[1] + bx[4]);
      const double pxt = near_image(xt, cx, ca.nx);
      const double pyt = ca.wall_y ? yt : near_image(yt, cy, ca.ny);
      const double hd = 0.5 * TILE2 * 1.41421356237309515;
      // whole tile outside the grown box: nothing to add (uniform branch)
      if (pxt + hd < bx[0] - reach || pxt - hd > bx[3] + reach || pyt + hd < bx[1] - reach ||
          pyt - hd > bx[4] + reach)
        continue;
      const double px = near_image((double)x, cx, ca.nx);
      const double py = ca.wall_y ? (double)y : near_image((double)y, cy, ca.ny);
      const bool inbox = px >= bx[0] - reach && px <= bx[3] + reach && py >= bx[1] - reach &&
                         py <= bx[4] + reach;
      double d2;
      int seg, inside;
      double tt;
      ring_geometry<NT>(md, ca, m, pxt, pyt, px, py, valid && inbox, d2, seg, tt, inside, s_cand,
                        s_int, s_dbl);
      if (valid && inbox) {
        const double d = sqrt(d2);
        if (d > ca.r_cut)
          Itot += inside ? 1.0 : 0.0;
        else
          Itot += 0.5 * (1.0 + tanh((inside ? d : -d) / (2.0 * ca.alpha)));
      }
    }
    const long long node = (long long)y * ca.nx + x;
    if (valid) Ifield[node] = Itot;
    if (!ca.want_force) continue;
    // pass 2: coupling force on the markers, -dE_c/dX (eq. DiscreteCF)
    double psi = 0.0;
    if (valid) {
      // psi(t) = sum_i h_i(x, t) by pull streaming of the current buffer
      using L = Lattice<9>;
      psi = cur.rest(2, node);
      for (int i = 1; i < 9; i++) {
        const int sy = y - L::cy[i];
        long long sn;
        int dir = i;
        if (ca.wall_y && (sy < 0 || sy >= ca.ny)) {
          sn = node;
          dir = L::opp[i];
        } else {
          sn = (long long)wrap(sy, ca.ny) * ca.nx + wrap(x - L::cx[i], ca.nx);
        }
        psi += (double)cur.template load<R>(2, dir, sn);
      }
    }
    for (int m = 0; m < md.K; m++) {
      const double* bx = md.mbox + 6 * m;
      const double cx = 0.5 * (bx[0] + bx[3]), cy = 0.5 * (bx[1] + bx[4]);
      const double pxt = near_image(xt, cx, ca.nx);
      const double pyt = ca.wall_y ? yt : near_image(yt, cy, ca.ny);
      const double hd = 0.5 * TILE2 * 1.41421356237309515;
      if (pxt + hd < bx[0] - reach || pxt - hd > bx[3] + reach || pyt + hd < bx[1] - reach ||
          pyt - hd > bx[4] + reach)
        continue;
      const double px = near_image((double)x, cx, ca.nx);
      const double py = ca.wall_y ? (double)y : near_image((double)y, cy, ca.ny);
      const bool inbox = px >= bx[0] - reach && px <= bx[3] + reach && py >= bx[1] - reach &&
                         py <= bx[4] + reach;
      double d2;
      int seg, inside;
      double tt;
      ring_geometry<NT>(md, ca, m, pxt, pyt, px, py, valid && inbox, d2, seg, tt, inside, s_cand,
                        s_int, s_dbl);
      if (!(valid && inbox) || seg < 0) continue;
      const double d = sqrt(d2);
      if (d > ca.r_cut || d == 0.0) continue;
      const int b = md.moff[m], n = md.moff[m + 1] - b;
      const int s1 = (seg + 1 == n) ? 0 : seg + 1;
      const double* X = md.X + 3 * b;
      const double fx = X[3 * seg] + tt * (X[3 * s1] - X[3 * seg]);
      const double fy = X[3 * seg + 1] + tt * (X[3 * s1 + 1] - X[3 * seg + 1]);
      const double nxh = (px - fx) / d, nyh = (py - fy) / d;
      const double sg = inside ? 1.0 : -1.0;
      const double ch = cosh((inside ? d : -d) / (2.0 * ca.alpha));
      const double wgt = ca.kappa_c / (4.0 * ca.alpha) * (psi - Itot) / (ch * ch);
      // dd/dX_vertex = -sign(d) nhat * barycentric weight
      const double gx = -sg * nxh * wgt, gy = -sg * nyh * wgt;
      long long* A = md.Facc + 3 * (b + seg);
      long long* B = md.Facc + 3 * (b + s1);
      atomicAdd((unsigned long long*)&A[0], (unsigned long long)to_fix(gx * (1.0 - tt)));
      atomicAdd((unsigned long long*)&A[1], (unsigned long long)to_fix(gy * (1.0 - tt)));
      atomicAdd((unsigned long long*)&B[0], (unsigned long long)to_fix(gx * tt));
      atomicAdd((unsigned long long*)&B[1], (unsigned long long)to_fix(gy * tt));
    }
  }
}

// ---------------------------------------------------------------------------
// ring strain + bending forces, gathered per marker (deterministic)

// bending energy term of vertex m: e = kb theta^2 / (|a| + |b|) with
// a = X_{m+1} - X_m, b = X_m - X_{m-1}, theta = atan2(a x b, a . b), i.e.
// (kb/4) (2 arccos y)^2 / ds' of eqs. DiscreteBE, DiscreteTheta,
// DiscreteArcLength.  Returns de/da and de/db.
__device__ __forceinline__ void bend_grad(double ax, double ay, double bx, double by, double kb,
                                          double& gax, double& gay, double& gbx, double& gby,
                                          double& e) {
  const double la2 = ax * ax + ay * ay, lb2 = bx * bx + by * by;
  const double la = sqrt(la2), lb = sqrt(lb2);
  const double cr = ax * by - ay * bx, dt = ax * bx + ay * by;
  const double th = atan2(cr, dt);
  const double L = la + lb;
  e = kb * th * th / L;
  // d theta = (dt d cr - cr d dt) / (|a|^2 |b|^2)
  const double inv = 1.0 / (la2 * lb2);
  const double tax = (dt * by - cr * bx) * inv, tay = (-dt * bx - cr * by) * inv;
  const double tbx = (-dt * ay - cr * ax) * inv, tby = (dt * ax - cr * ay) * inv;
  const double c1 = 2.0 * kb * th / L, c2 = kb * th * th / (L * L);
  gax = c1 * tax - c2 * ax / la;
  gay = c1 * tay - c2 * ay / la;
  gbx = c1 * tbx - c2 * bx / lb;
  gby = c1 * tby - c2 * by / lb;
}

__global__ void k_memforce2d(MemDev md) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= md.M) return;
  const int m = md.mid[g];
  const int b = md.moff[m], n = md.moff[m + 1] - b;
  const int l = g - b;
  auto P = [&](int k, int a) { return md.X[3 * (b + ((l + k) % n + n) % n) + a]; };
  auto rest = [&](int k) { return md.rest[b + ((l + k) % n + n) % n]; };
  const double ks = md.ks[m], kbm = md.kb[m];
  double Fx = 0, Fy = 0;
  // strain, eq. DiscreteSF: segments l-1 -> l and l -> l+1
  {
    const double ex = P(1, 0) - P(0, 0), ey = P(1, 1) - P(0, 1);
    const double len = sqrt(ex * ex + ey * ey);
    const double s = ks * (len / rest(0) - 1.0) / len;
    Fx += s * ex;
    Fy += s * ey;
    const double fx = P(0, 0) - P(-1, 0), fy = P(0, 1) - P(-1, 1);
    const double lf = sqrt(fx * fx + fy * fy);
    const double sf = ks * (lf / rest(-1) - 1.0) / lf;
    Fx -= sf * fx;
    Fy -= sf * fy;
  }
  // bending, eq. DiscreteBF: vertex terms l-1, l, l+1 depend on X_l
  if (kbm != 0.0) {
    double gax, gay, gbx, gby, e;
    // vertex l-1: X_l = X_{(l-1)+1} enters through a
    bend_grad(P(0, 0) - P(-1, 0), P(0, 1) - P(-1, 1), P(-1, 0) - P(-2, 0), P(-1, 1) - P(-2, 1), kbm,
              gax, gay, gbx, gby, e);
    Fx -= gax;
    Fy -= gay;
    // vertex l: a = X_{l+1} - X_l (dX_l: -1), b = X_l - X_{l-1} (dX_l: +1)
    bend_grad(P(1, 0) - P(0, 0), P(1, 1) - P(0, 1), P(0, 0) - P(-1, 0), P(0, 1) - P(-1, 1), kbm, gax,
              gay, gbx, gby, e);
    Fx -= -gax + gbx;
    Fy -= -gay + gby;
    // vertex l+1: X_l = X_{(l+1)-1} enters through b with sign -1
    bend_grad(P(2, 0) - P(1, 0), P(2, 1) - P(1, 1), P(1, 0) - P(0, 0), P(1, 1) - P(0, 1), kbm, gax,
              gay, gbx, gby, e);
    Fx += gbx;
    Fy += gby;
  }
  // coupling force accumulated by the profile kernel
  long long* acc = md.Facc + 3 * g;
  Fx += from_fix(acc[0]);
  Fy += from_fix(acc[1]);
  acc[0] = 0;
  acc[1] = 0;
  acc[2] = 0;
  if (!(fabs(Fx) < FIX_LIMIT) || !(fabs(Fy) < FIX_LIMIT)) md.status[0] = 1;
  md.F[3 * g] = Fx;
  md.F[3 * g + 1] = Fy;
  md.F[3 * g + 2] = 0.0;
}

// spreading, eq. Spreading with delta x = 1 (READING: no extra Delta s): each
// marker adds F delta_h(x - X) to its 16 stencil nodes in fixed point
__global__ void k_spread2d(MemDev md, long long* __restrict__ fib, int nx, int ny, int wall_y) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= md.M) return;
  const double X = md.X[3 * g], Y = md.X[3 * g + 1];
  const double Fx = md.F[3 * g], Fy = md.F[3 * g + 1];
  const int bx = (int)floor(X) - 1, by = (int)floor(Y) - 1;
  double wx[4], wy[4];
  for (int k = 0; k < 4; k++) {
    wx[k] = peskin((bx + k) - X);
    wy[k] = peskin((by + k) - Y);
  }
  for (int ky = 0; ky < 4; ky++) {
    const int yy = by + ky;
    if (wall_y && (yy < 0 || yy >= ny)) continue;
    const int yw = wrap(yy, ny);
    for (int kx = 0; kx < 4; kx++) {
      const double w = wx[kx] * wy[ky];
      const long long node = (long long)yw * nx + wrap(bx + kx, nx);
      atomicAdd((unsigned long long*)&fib[2 * node], (unsigned long long)to_fix(Fx * w));
      atomicAdd((unsigned long long*)&fib[2 * node + 1], (unsigned long long)to_fix(Fy * w));
    }
  }
}

// interpolation of v* = u(t+1) + f(t) / (2 rho(t+1)) at the stencil of X(t)
// (eq. Interpolation, READING: the force of step t stands in for the unknown
// force at t+1), then X(t+1) = X(t) + U (eq. UpdatedXl)
template <class St, typename R>
__global__ void k_interp2d(MemDev md, St cur, LBParams P, const double* __restrict__ force) {
  using L = Lattice<9>;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= md.M) return;
  const double X = md.X[3 * g], Y = md.X[3 * g + 1];
  const int bx = (int)floor(X) - 1, by = (int)floor(Y) - 1;
  double wx[4], wy[4];
  for (int k = 0; k < 4; k++) {
    wx[k] = peskin((bx + k) - X);
    wy[k] = peskin((by + k) - Y);
  }
  double Ux = 0, Uy = 0;
  for (int ky = 0; ky < 4; ky++) {
    const int yy = by + ky;
    if (P.wall_y && (yy < 0 || yy >= P.ny)) continue;
    const int yw = wrap(yy, P.ny);
    for (int kx = 0; kx < 4; kx++) {
      const int xw = wrap(bx + kx, P.nx);
      const long long node = (long long)yw * P.nx + xw;
      double d = 0, jx = 0, jy = 0;
      for (int i = 0; i < 9; i++) {
        const int sy = yw - L::cy[i];
        long long sn;
        int dir = i;
        if (P.wall_y && (sy < 0 || sy >= P.ny)) {
          sn = node;
          dir = L::opp[i];
        } else {
          sn = (long long)wrap(sy, P.ny) * P.nx + wrap(xw - L::cx[i], P.nx);
        }
        const double v = (double)cur.template load<R>(0, dir, sn);
        d += v;
        jx += L::cx[i] * v;
        jy += L::cy[i] * v;
      }
      const double rho = 1.0 + d;
      const double vx = (jx + 0.5 * force[2 * node]) / rho;
      const double vy = (jy + 0.5 * force[2 * node + 1]) / rho;
      const double w = wx[kx] * wy[ky];
      Ux += vx * w;
      Uy += vy * w;
    }
  }
  md.U[3 * g] = Ux;
  md.U[3 * g + 1] = Uy;
  md.U[3 * g + 2] = 0.0;
  md.X[3 * g] = X + Ux;
  md.X[3 * g + 1] = Y + Uy;
}

}  // namespace lb
