// k_ibm.h -- membrane side of the step for 2D ring membranes: active-tile
// map, coupling profile I and coupling force (Sec. 2.5 eq. Iprofile, Sec. 3.2
// eqs. DiscreteCE/DiscreteCF), strain and bending forces (eqs. DiscreteSF,
// DiscreteBF), spreading (eq. Spreading) and interpolation + Euler update
// (eqs. Interpolation, UpdatedXl).  All marker arithmetic is FP64.
//
// Active tiles: every lattice tile (TILE x TILE nodes) that meets a
// membrane's bounding box grown by map_reach(r_cut).  Only these tiles carry a
// profile I different from 0, a spread force, or a stored total force; the
// fused lattice kernel reads the maps there and nowhere else.  A tile is
// active in a step when its flag equals that step's stamp, so no pass is
// needed to clear the previous step's map.
//
// Signed distance d(x): distance to the closest segment of the marker
// polygon, positive inside.  Every node of a tile is compared with all
// segments within reach of the tile (enough to contain each node's closest
// segment); the sign comes from the closest feature: the side of the closest
// segment, or at a closest vertex the sum of its two edge normals (exact for
// a simple polygon, whichever way it is oriented).
#pragma once
#include "common.h"
#include "k_lb.h"

namespace lb {

constexpr int TILE2 = 16;          // 2D tile edge
constexpr int COUP_THREADS = 256;  // one thread per node of a 16x16 tile
constexpr int COUP_CHUNK = 512;    // segments examined per culling chunk
constexpr int COUP_KEEP = 4;       // membranes per tile whose band data stays in LDS
constexpr int COUP_ML = 64;        // membranes whose grown boxes may meet one tile
constexpr int COUP_CACHE = 2;      // membranes per tile whose closest segment each node keeps
// with the cache on, the candidate lists reach this much farther: every
// segment left off a node's list is then at least this much farther than
// its closest one, the room a cached entry has before the markers' drift
// expires it
constexpr float COUP_PAD = 2.0f;
constexpr int COUP_WIN = 8;        // a cached entry re-evaluates its segment and 8 on each side
// a wave renews at most this many expired entries one by one (each costs a
// pass over the whole ring, about what the tile's full search costs its
// nodes); with more, the tile searches in full and renews every entry
constexpr int COUP_RENEW = 8;
// with the cache on, a tile, sub-tile or node is taken to lie beyond the
// band without a search only this much farther out, so its entry outlasts
// some drift; nearer nodes are searched and keep their closest segment
constexpr float COUP_BEYOND = 1.0f;
constexpr int COUP_FACC = 128;     // per-tile LDS accumulator of coupling forces, markers per slot

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
  int* law;           // K, strain law of each 2D ring (0 eq. DiscreteSE, 1 neo-Hookean, 2 Skalak)
  double* mbox;       // 8 per membrane: lo xyz, hi xyz, orientation (+-1), drift: a bound on
                      // the distance any marker has moved since the simulation started
  int* status;        // [0] force/marker out of range, [1] lattice too small / too many membranes
  float4* stab;       // 2D, per step: segment l -> l+1 as (start - box centre, edge) in FP32
  float* sinv;        // 2D, per step: 1 / |edge|^2
  int K, M;
};

struct TileMap {
  int* tflag;         // per tile: stamp of the last step it was active in
  int* tlist;         // active tiles of this step
  int* tstate;        // [0] active-tile count, [1] stamp of this step, [2] 3D tile counter,
                      // [4], [5] active-tile counts of a 2D simulation, by stamp parity
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
  for (int i = 0; i < NT / 64; i++) t += sh[i];
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
  double t = sh[0];
  for (int i = 1; i < NT / 64; i++) t = fmin(t, sh[i]);
  __syncthreads();
  return t;
}

// seven minima and one sum over the block with a single exchange, in the
// order of block_min and block_sum (bitwise the same results)
template <int NT>
__device__ void block_min7_sum1(double (&v)[8], double* sh) {
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < 7; k++) v[k] = fmin(v[k], __shfl_down(v[k], o, 64));
    v[7] += __shfl_down(v[7], o, 64);
  }
  constexpr int W = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 8; k++) sh[k * W + wv] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 7; k++) {
    double t = sh[k * W];
    for (int i = 1; i < W; i++) t = fmin(t, sh[k * W + i]);
    v[k] = t;
  }
  double t = 0;
  for (int i = 0; i < W; i++) t += sh[7 * W + i];
  v[7] = t;
  __syncthreads();
}

__device__ __forceinline__ float wave_minf(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NT>
__device__ float block_minf(float v, float* sh) {
  v = wave_minf(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  float t = sh[0];
  for (int k = 1; k < NT / 64; k++) t = fminf(t, sh[k]);
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// new step of the tile map (3D simulations and batch members; one thread):
// [0] active-tile count, [1] stamp, [2] counter the 3D profile kernel's
// workgroups take tiles from
__global__ void k_begin(int* tstate) {
  if (threadIdx.x == 0) {
    tstate[0] = 0;
    tstate[1] = tstate[1] + 1;
    tstate[2] = 0;
  }
}

// bounding box, orientation and active tiles of membrane blockIdx.x
template <int NT>
__device__ __forceinline__ void tiles_run(const MemDev& md, const TileMap& tm, int nx, int ny, int nz,
                                          int wall_y, int wall_z, int D, double reach, int m, int stamp,
                                          int* __restrict__ cnt) {
  __shared__ double sh[8 * (NT / 64)];
  const int tid = threadIdx.x;
  const int b = md.moff[m], e = md.moff[m + 1], n = e - b;
  // one pass over the markers: box (minima of X and of -X), largest step of
  // the last marker update |U| (each step adds it to the membrane's drift
  // bound; a call between steps adds it again, which only loosens the bound)
  // and, in 2D, the signed area (shoelace sum) that gives the orientation;
  // then one block-wide exchange for all eight values
  double v[8] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300, 0.0, 0.0};
  for (int l = tid; l < n; l += NT) {
    const double* Xl = md.X + 3 * (b + l);
    for (int a = 0; a < D; a++) {
      v[a] = fmin(v[a], Xl[a]);
      v[3 + a] = fmax(v[3 + a], Xl[a]);
    }
    const double* Ul = md.U + 3 * (b + l);
    v[6] = fmax(v[6], Ul[0] * Ul[0] + Ul[1] * Ul[1] + Ul[2] * Ul[2]);
    if (D == 2) {
      const int l1 = (l + 1 == n) ? 0 : l + 1;
      const double* X1 = md.X + 3 * (b + l1);
      v[7] += Xl[0] * X1[1] - X1[0] * Xl[1];
    }
  }
  for (int k = 3; k < 7; k++) v[k] = -v[k];
  block_min7_sum1<NT>(v, sh);
  double lo[3], hi[3];
  for (int a = 0; a < 3; a++) {
    lo[a] = v[a];
    hi[a] = -v[3 + a];
  }
  const double umax = sqrt(-v[6]);
  const double area = D == 2 ? v[7] : 0.0;
  if (tid == 0) {
    for (int a = 0; a < 3; a++) {
      md.mbox[8 * m + a] = lo[a];
      md.mbox[8 * m + 3 + a] = hi[a];
    }
    // with room for the rounding of X + U
    md.mbox[8 * m + 7] += umax * (1.0 + 1e-12) + 1e-12;
    md.mbox[8 * m + 6] = area >= 0.0 ? 1.0 : -1.0;
  }
  // 2D: this step's FP32 segment table, relative to the box centre
  if (D == 2) {
    const double cx = 0.5 * (lo[0] + hi[0]), cy = 0.5 * (lo[1] + hi[1]);
    for (int l = tid; l < n; l += NT) {
      const int g = b + l, g1 = (l + 1 == n) ? b : g + 1;
      const double ex = md.X[3 * g1] - md.X[3 * g], ey = md.X[3 * g1 + 1] - md.X[3 * g + 1];
      const double ee = ex * ex + ey * ey;
      md.stab[g] = make_float4((float)(md.X[3 * g] - cx), (float)(md.X[3 * g + 1] - cy), (float)ex, (float)ey);
      md.sinv[g] = ee > 0.0 ? (float)(1.0 / ee) : 0.0f;
    }
  }
  // non-finite or runaway markers: flag and leave this membrane off the map
  for (int a = 0; a < D; a++)
    if (!(fabs(lo[a]) < 1e9) || !(fabs(hi[a]) < 1e9)) {
      if (tid == 0) md.status[0] = 1;
      return;
    }
  const int dims[3] = {nx, ny, nz};
  const int per[3] = {1, !wall_y, !wall_z};
  // the grown box must be narrower than the period: the band of a membrane
  // may not reach around the lattice onto itself
  for (int a = 0; a < D; a++)
    if (per[a] && hi[a] - lo[a] + 2.0 * reach >= dims[a] && tid == 0) md.status[1] = 1;
  int t0[3] = {0, 0, 0}, t1[3] = {0, 0, 0};
  const int nt[3] = {tm.ntx, tm.nty, tm.ntz};
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
  if (sx <= 0 || sy <= 0 || sz <= 0) return;
  const long long total = (long long)sx * sy * sz;
  for (long long q = tid; q < total; q += NT) {
    const int ix = (int)(q % sx), iy = (int)((q / sx) % sy), iz = (int)(q / ((long long)sx * sy));
    const int tx = wrap(t0[0] + ix, nt[0]), ty = wrap(t0[1] + iy, nt[1]);
    const int tz = (D == 3) ? wrap(t0[2] + iz, nt[2]) : 0;
    const int t = (tz * tm.nty + ty) * tm.ntx + tx;
    // a tile first marked in this step takes a list slot: one counter
    // update per wave for all of its newly marked tiles
    const bool fresh = atomicMax(&tm.tflag[t], stamp) < stamp;
    const unsigned long long mk = __ballot(fresh);
    if (mk) {
      const int lane = tid & 63, lead = __ffsll((long long)mk) - 1;
      int base = 0;
      if (lane == lead) base = atomicAdd(cnt, __popcll(mk));
      base = __shfl(base, lead, 64);
      if (fresh) tm.tlist[base + __popcll(mk & ((1ull << lane) - 1ull))] = t;
    }
  }
}

// stamp > 0: this pass's stamp, chosen by the host (a 2D simulation); the
// tiles are counted in tstate[4 + (stamp & 1)], and the first thread
// publishes the stamp and empties the other counter for the next pass.
// stamp 0: the stamp and the empty counter tstate[0] that k_begin prepared.
template <int NT>
__global__ __launch_bounds__(NT) void k_tiles(MemDev md, TileMap tm, int nx, int ny, int nz,
                                              int wall_y, int wall_z, int D, double reach, int stamp) {
  int* cnt = tm.tstate;
  if (stamp > 0) {
    cnt = tm.tstate + 4 + (stamp & 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      tm.tstate[1] = stamp;
      tm.tstate[4 + ((stamp + 1) & 1)] = 0;
    }
  } else {
    stamp = tm.tstate[1];
  }
  tiles_run<NT>(md, tm, nx, ny, nz, wall_y, wall_z, D, reach, (int)blockIdx.x, stamp, cnt);
}

// FP32 squared distance from p to the segment (s.x, s.y) + t (s.z, s.w)
__device__ __forceinline__ float seg_d2f(float px, float py, float4 sg, float inv) {
  const float qx = px - sg.x, qy = py - sg.y;
  const float t = fminf(fmaxf((qx * sg.z + qy * sg.w) * inv, 0.0f), 1.0f);
  const float dx = qx - t * sg.z, dy = qy - t * sg.w;
  return dx * dx + dy * dy;
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

__device__ __forceinline__ double near_image(double v, double c, int n) {
  return v + n * floor((c - v) / n + 0.5);
}

struct CoupArgs {
  int nx, ny, wall_y;
  double alpha, kappa_c, r_cut;
  int want_force;
  // per node and cached membrane slot (COUP_CACHE x N): the membrane and
  // closest segment of the last full search (key = m << 16 | segment, or
  // m << 16 | 0xFFFE / 0xFFFD for a node beyond the band inside / outside;
  // -1 none), and a lower bound (plus the membrane's drift at that time) on
  // the distance of every segment more than COUP_WIN from the closest one
  // (beyond the band: on the distance of the ring); null disables the cache
  int* ckey;
  float* clb;
  long long N;
};

// inside test at the closest feature of a ring (markers X, n of them,
// orientation o = +1 counter-clockwise): the side of segment s at parameter
// t, or at an end vertex the side of the sum of the two edge normals;
// (ax, ay) and (bx, by) are the end points of s, already loaded
__device__ __forceinline__ bool ring_side_ab(const double* X, int n, double o, int s, double t, double ax,
                                             double ay, double bx, double by, double px, double py) {
  const int s1 = (s + 1 == n) ? 0 : s + 1;
  if (t > 0.0 && t < 1.0) return o * ((bx - ax) * (py - ay) - (by - ay) * (px - ax)) > 0.0;
  // the closest point is a vertex v: its edges from the previous vertex u
  // and to the next w (one of them is the segment itself)
  double vx, vy, ux, uy, wx, wy;
  if (t <= 0.0) {
    const int u = (s == 0) ? n - 1 : s - 1;
    vx = ax, vy = ay, wx = bx, wy = by;
    ux = X[3 * u], uy = X[3 * u + 1];
  } else {
    const int w = (s1 + 1 == n) ? 0 : s1 + 1;
    vx = bx, vy = by, ux = ax, uy = ay;
    wx = X[3 * w], wy = X[3 * w + 1];
  }
  const double e1x = vx - ux, e1y = vy - uy;
  const double e2x = wx - vx, e2y = wy - vy;
  const double l1 = sqrt(e1x * e1x + e1y * e1y), l2 = sqrt(e2x * e2x + e2y * e2y);
  // left normals (-ey, ex) of both edges, summed
  const double nx_ = -e1y / l1 - e2y / l2, ny_ = e1x / l1 + e2x / l2;
  return o * (nx_ * (px - vx) + ny_ * (py - vy)) > 0.0;
}

__device__ __forceinline__ bool ring_side(const double* X, int n, double o, int s, double t, double px,
                                          double py) {
  const int s1 = (s + 1 == n) ? 0 : s + 1;
  return ring_side_ab(X, n, o, s, t, X[3 * s], X[3 * s + 1], X[3 * s1], X[3 * s1 + 1], px, py);
}

// How far beyond a membrane's box the tile map reaches (2D and 3D): the
// coupling pass takes a membrane for a tile within r_cut + 1 of its box
// (beyond, the profile is 0 and no force arises), and spreading writes up to
// two nodes beyond the markers, which the lattice kernels read on mapped
// tiles only.
__host__ __device__ __forceinline__ double map_reach(double r_cut) { return fmax(r_cut + 1.0, 3.0); }

// profile value 0.5 (1 + tanh x) of eq. Iprofile (x = d / (2 alpha), d the
// signed distance) and sech^2 x, the factor of the coupling force (eq.
// DiscreteCF), from one exponential
__device__ __forceinline__ double profile_sech2(double x, double& s2) {
  const double em = expm1(-2.0 * fabs(x));  // e^{-2|x|} - 1, in (-1, 0]
  const double th = -em / (2.0 + em);        // tanh |x|
  s2 = 4.0 * (1.0 + em) / ((2.0 + em) * (2.0 + em));
  return 0.5 * (1.0 + (x < 0.0 ? -th : th));
}

// A band node at signed distance sd (|sd| = d) from the closest point of
// the segment from a to b (parameter t): the direction in which the coupling
// energy pushes the segment's vertices, -sign(sd) nhat sech^2(sd / (2 alpha))
// with nhat the unit vector from the closest point to the node (eq.
// DiscreteCF without the factor kappa_c / (4 alpha) (psi - I) and the vertex
// weights).  Zero for a node on the ring, where nhat is undefined.
__device__ __forceinline__ void band_push(double ax, double ay, double bx, double by, double t, double px,
                                          double py, double sd, double s2, double& gx, double& gy) {
  const double d = fabs(sd);
  gx = gy = 0.0;
  if (d == 0.0) return;
  const double fx = ax + t * (bx - ax);
  const double fy = ay + t * (by - ay);
  const double sg = sd > 0.0 ? 1.0 : -1.0;
  gx = -sg * ((px - fx) / d) * s2;
  gy = -sg * ((py - fy) / d) * s2;
}

// do the nodes of the tile starting at s (width TILE2, lattice n) fall into
// different periodic images relative to centre c?  (the tile straddles the
// antipode of c; its nodes are then searched one by one)
__device__ __forceinline__ bool tile_splits(int s, int n, double c) {
  const int e = min(s + TILE2 - 1, n - 1);
  return near_image((double)s, c, n) - s != near_image((double)e, c, n) - e;
}

// exact FP64 closest segment to (px, py) among the candidates of a wave list
// whose FP32 value lies within tol of the FP32 minimum bf, reduced over the
// wave (lowest segment index on equal distances); every lane gets the result
__device__ __forceinline__ void wave_closest(const unsigned short* wl, int cnt, const int* cand,
                                             const float4* geo, const float* inv, const double4* end,
                                             float fx, float fy, float bf, double px, double py, double& d2b,
                                             int& sb, double& tb) {
  const float tol = 2e-3f + 2e-5f * bf;
  d2b = 1e300;
  sb = 0x7fffffff;
  tb = 0.0;
  for (int k = (int)(threadIdx.x & 63); k < cnt; k += 64) {
    const int q = wl[k];
    const float4 g4 = geo[q];
    const float qx = fx - g4.x, qy = fy - g4.y;
    const float sp = fminf(fmaxf((qx * g4.z + qy * g4.w) * inv[q], 0.0f), 1.0f);
    const float dx = qx - sp * g4.z, dy = qy - sp * g4.w;
    if (dx * dx + dy * dy > bf + tol) continue;
    const double4 e = end[q];
    double tt;
    const double d2 = seg_d2(px, py, e.x, e.y, e.z, e.w, tt);
    const int s = cand[q];
    if (d2 < d2b || (d2 == d2b && s < sb)) {
      d2b = d2;
      sb = s;
      tb = tt;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double d2o = __shfl_xor(d2b, o, 64), to = __shfl_xor(tb, o, 64);
    const int so = __shfl_xor(sb, o, 64);
    if (d2o < d2b || (d2o == d2b && so < sb)) {
      d2b = d2o;
      sb = so;
      tb = to;
    }
  }
}

// one active tile li of the list, all NT threads of the workgroup
template <class St, typename R, int NT>
__device__ __forceinline__ void coupling2d_tile(const MemDev& md, const TileMap& tm, const CoupArgs& ca,
                                                double* __restrict__ Ifield, const St& cur, int li) {
  static_assert(NT == TILE2 * TILE2, "one thread per node of a tile");
  __shared__ int s_cand[COUP_CHUNK];
  __shared__ float4 s_geo[COUP_CHUNK];  // candidate start point and edge, relative to the tile centre
  __shared__ float s_inv[COUP_CHUNK];   // 1 / |edge|^2
  __shared__ double4 s_end[COUP_CHUNK]; // candidate end points X_s, X_s+1 in FP64
  __shared__ unsigned short s_wl[NT / 64][COUP_CHUNK];  // per-wave candidate lists
  __shared__ int s_cnt;
  __shared__ double s_red[NT / 64];
  __shared__ float s_redf[NT / 64];
  __shared__ int s_ml[COUP_ML];  // membranes whose grown box meets the tile, ascending
  __shared__ double s_mbx[COUP_ML][8];  // their boxes (the eight words of mbox)
  __shared__ int s_mof[COUP_ML][2];     // and marker ranges [moff[m], moff[m + 1])
  __shared__ int s_mn, s_wc[NT / 64];
  __shared__ long long s_facc[COUP_FACC][2];  // coupling forces of one slot's markers, fixed point
  __shared__ int s_base;
  __shared__ int b_seg[COUP_KEEP][NT];
  __shared__ double b_t[COUP_KEEP][NT];
  __shared__ double b_gx[COUP_KEEP][NT];  // band_push direction of each band node
  __shared__ double b_gy[COUP_KEEP][NT];
  const double reach = ca.r_cut + 1.0;
  const double hd = 0.5 * TILE2 * 1.41421356237309515;
  {
    const int t = tm.tlist[li];
    const int tx = t % tm.ntx, ty = t / tm.ntx;
    // wave w holds the 8 x 8 sub-tile (w & 1, w >> 1) of the 16 x 16 tile
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = tx * TILE2 + (wv & 1) * 8 + (lane & 7), y = ty * TILE2 + (wv >> 1) * 8 + (lane >> 3);
    // sub-tile centre relative to the tile centre
    const float cwx = (wv & 1) ? 4.0f : -4.0f, cwy = (wv >> 1) ? 4.0f : -4.0f;
    const unsigned long long below = (1ull << lane) - 1ull;
    // largest distance of a node from its tile / sub-tile centre
    const double rn16 = 7.5 * 1.41421356237309515, rn8 = 3.5 * 1.41421356237309515;
    const bool valid = (x < ca.nx) && (y < ca.ny);
    const long long node = (long long)y * ca.nx + x;
    // The boxes of the first NT membranes, for the list below, are loaded
    // first; then the loads that depend on the node only, whose latency the
    // list overlaps: the cache entries of the first COUP_CACHE slots and, for
    // the force, the populations h_i that sum to psi.  Every lane issues all
    // of them (indices clamped: a lane past the lattice edge, or without the
    // cache, reads a valid location whose value it never uses), so the list
    // waits for the boxes alone: waits count outstanding loads in issue order.
    const int mq = min((int)threadIdx.x, md.K - 1);
    double mbq[8];
#pragma unroll
    for (int k = 0; k < 8; k++) mbq[k] = md.mbox[8 * mq + k];
    const int mo0 = md.moff[mq], mo1 = md.moff[mq + 1];
    asm volatile("" ::: "memory");
    const int xc = min(x, ca.nx - 1), yc = min(y, ca.ny - 1);
    const long long cnode = (long long)yc * ca.nx + xc;
    int kpre[COUP_CACHE];
    float lpre[COUP_CACHE];
    {
      const bool on = ca.ckey != nullptr;
      const int* kp = on ? ca.ckey : md.status;
      const float* lp = on ? ca.clb : (const float*)md.status;
#pragma unroll
      for (int c = 0; c < COUP_CACHE; c++) {
        const long long e = on ? (long long)c * ca.N + cnode : 0;
        kpre[c] = kp[e];
        lpre[c] = lp[e];
      }
    }
    R hmov[8];
    const double hrest = cur.rest(2, cnode);
    {
      using L = Lattice<9>;
      // neighbour rows and columns of (xc, yc), wrapped once
      const long long rlo = (long long)(yc == 0 ? ca.ny - 1 : yc - 1) * ca.nx;
      const long long rhi = (long long)(yc == ca.ny - 1 ? 0 : yc + 1) * ca.nx;
      const int xlo = xc == 0 ? ca.nx - 1 : xc - 1, xhi = xc == ca.nx - 1 ? 0 : xc + 1;
      const bool wlo = ca.wall_y && yc == 0, whi = ca.wall_y && yc == ca.ny - 1;
#pragma unroll
      for (int i = 1; i < 9; i++) {
        const bool back = L::cy[i] > 0 ? wlo : (L::cy[i] < 0 ? whi : false);
        const long long row = L::cy[i] > 0 ? rlo : (L::cy[i] < 0 ? rhi : cnode - xc);
        const int col = L::cx[i] > 0 ? xlo : (L::cx[i] < 0 ? xhi : xc);
        hmov[i - 1] = cur.template load<R>(2, back ? L::opp[i] : i, back ? cnode : row + col);
      }
    }
    const double xt = tx * TILE2 + 0.5 * (TILE2 - 1), yt = ty * TILE2 + 0.5 * (TILE2 - 1);
    // image of the tile centre nearest a membrane's box centre (cx, cy): the
    // image of the tile's first node, since the nodes of a tile that does
    // not split share one image.  (The nominal centre of a partial tile at
    // the lattice edge can lie beyond the antipode while its nodes do not.)
    auto tile_image = [&](double cx, double cy, double& pxt, double& pyt) {
      pxt = xt + (near_image((double)(tx * TILE2), cx, ca.nx) - tx * TILE2);
      pyt = ca.wall_y ? yt : yt + (near_image((double)(ty * TILE2), cy, ca.ny) - ty * TILE2);
    };
    // Per axis, the grown box [lo - reach, hi + reach] against the tile: the
    // square of half-width hd around the tile centre's image, or, when the
    // tile's nodes fall into two images (it straddles the antipode of the box
    // centre c), each image's run of nodes: from the first node's image up to
    // c + n/2, and from c - n/2 up to the last node's image (the grown box is
    // narrower than the period, so it reaches neither c + n/2 nor c - n/2).
    auto axis_meets = [&](int s0, int n, double c, double lo, double hi, double pt, bool split) {
      if (split) {
        const int e = min(s0 + TILE2 - 1, n - 1);
        return near_image((double)s0, c, n) <= hi + reach || near_image((double)e, c, n) >= lo - reach;
      }
      return !(pt + hd < lo - reach || pt - hd > hi + reach);
    };
    auto meets_box = [&](double b0, double b1, double b3, double b4) {
      const double cx = 0.5 * (b0 + b3), cy = 0.5 * (b1 + b4);
      double pxt, pyt;
      tile_image(cx, cy, pxt, pyt);
      const bool sx = tile_splits(tx * TILE2, ca.nx, cx);
      const bool sy = !ca.wall_y && tile_splits(ty * TILE2, ca.ny, cy);
      return axis_meets(tx * TILE2, ca.nx, cx, b0, b3, pxt, sx) && axis_meets(ty * TILE2, ca.ny, cy, b1, b4, pyt, sy);
    };
    // the membranes this tile meets, tested in parallel and listed in
    // ascending order (ordered compaction by ballots)
    if (threadIdx.x == 0) s_mn = 0;
    __syncthreads();
    for (int c0 = 0; c0 < md.K; c0 += NT) {
      const int m = c0 + threadIdx.x;
      double bv[8];
      int ov[2];
      if (c0 == 0) {
#pragma unroll
        for (int k = 0; k < 8; k++) bv[k] = mbq[k];
        ov[0] = mo0;
        ov[1] = mo1;
      } else if (m < md.K) {
#pragma unroll
        for (int k = 0; k < 8; k++) bv[k] = md.mbox[8 * m + k];
        ov[0] = md.moff[m];
        ov[1] = md.moff[m + 1];
        // (more than NT membranes) these loads complete here, so that no
        // wait after the list has to cover the node's loads issued above
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      }
      const bool mt = m < md.K && meets_box(bv[0], bv[1], bv[3], bv[4]);
      const unsigned long long mk = __ballot(mt);
      if (lane == 0) s_wc[wv] = __popcll(mk);
      __syncthreads();
      int off = s_mn, tot = 0;
      for (int w = 0; w < NT / 64; w++) {
        off += w < wv ? s_wc[w] : 0;
        tot += s_wc[w];
      }
      const int pos = off + __popcll(mk & below);
      if (mt && pos < COUP_ML) {
        s_ml[pos] = m;
#pragma unroll
        for (int k = 0; k < 8; k++) s_mbx[pos][k] = bv[k];
        s_mof[pos][0] = ov[0];
        s_mof[pos][1] = ov[1];
      }
      __syncthreads();
      if (threadIdx.x == 0) s_mn += tot;
      __syncthreads();
    }
    const int nm = s_mn;
    if (nm > COUP_ML && threadIdx.x == 0) md.status[1] = 1;
    double Itot = 0.0;
    // a node farther than r_cut from a ring lies on the side of its
    // sub-tile centre (the segment between them meets no marker) when the
    // band is wider than a sub-tile's reach
    const bool shortcut = ca.r_cut > rn8 + 1.0;
    for (int slot = 0; slot < min(nm, COUP_ML); slot++) {
      const int m = s_ml[slot];
      const double* bx = s_mbx[slot];
      const double cx = 0.5 * (bx[0] + bx[3]), cy = 0.5 * (bx[1] + bx[4]);
      double pxt, pyt;
      tile_image(cx, cy, pxt, pyt);
      const bool split = tile_splits(tx * TILE2, ca.nx, cx) || (!ca.wall_y && tile_splits(ty * TILE2, ca.ny, cy));
      const int b = s_mof[slot][0], n = s_mof[slot][1] - b;
      const double* X = md.X + 3 * b;
      const double o = bx[6];
      const double px = near_image((double)x, cx, ca.nx);
      const double py = ca.wall_y ? (double)y : near_image((double)y, cy, ca.ny);
      const bool inbox = valid && px >= bx[0] - reach && px <= bx[3] + reach &&
                         py >= bx[1] - reach && py <= bx[4] + reach;
      if (split) {
        // nodes of different images: each one searches the whole ring
        double d2b = 1e300, tb = 0.0;
        int sb = -1;
        if (inbox)
          for (int l = 0; l < n; l++) {
            const int l1 = (l + 1 == n) ? 0 : l + 1;
            double tt;
            const double d2 = seg_d2(px, py, X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1], tt);
            if (d2 < d2b) {
              d2b = d2;
              sb = l;
              tb = tt;
            }
          }
        bool band = false;
        double gx = 0.0, gy = 0.0;
        if (inbox && sb >= 0) {
          const double d = sqrt(d2b);
          const int sb1 = (sb + 1 == n) ? 0 : sb + 1;
          const double eax = X[3 * sb], eay = X[3 * sb + 1], ebx = X[3 * sb1], eby = X[3 * sb1 + 1];
          const bool in = ring_side_ab(X, n, o, sb, tb, eax, eay, ebx, eby, px, py);
          const double sd = in ? d : -d;
          band = d <= ca.r_cut;
          if (band) {
            double s2;
            Itot += profile_sech2(sd / (2.0 * ca.alpha), s2);
            if (ca.want_force) band_push(eax, eay, ebx, eby, tb, px, py, sd, s2, gx, gy);
          } else {
            Itot += in ? 1.0 : 0.0;
          }
        }
        if (slot < COUP_KEEP) {
          b_seg[slot][threadIdx.x] = band ? sb : -1;
          b_t[slot][threadIdx.x] = tb;
          b_gx[slot][threadIdx.x] = gx;
          b_gy[slot][threadIdx.x] = gy;
        }
        continue;
      }
      double d2b = 1e300, tb = 0.0;
      int sb = -1;
      int side = -1;  // side of a node beyond the band (-1: not decided that way)
      // Temporal coherence.  A node keeps its closest segment s of the last
      // full search and a lower bound L on the distance of every segment
      // more than COUP_WIN away from s along the ring.  No marker has moved
      // farther than the membrane's drift since, and a segment's distance
      // moves no more than its end points, so while the nearest of the
      // segments within COUP_WIN of s (exact, in FP64, lowest index on ties)
      // is nearer than L less the drift, it is the closest segment a full
      // search would find.  A node beyond the
      // band stays beyond it, on its side, while its distance bound less
      // the drift exceeds r_cut.  The tile skips the search when every
      // node is certified.
      const bool cslot = ca.ckey != nullptr && slot < COUP_CACHE && n <= COUP_CHUNK && m < 32768;
      const long long cix = (long long)slot * ca.N + ((long long)y * ca.nx + x);
      bool cached = false;
      if (cslot) {
        bool ok = true;
        int key = kpre[0];
        float klb = lpre[0];
#pragma unroll
        for (int c = 1; c < COUP_CACHE; c++)
          if (slot == c) {
            key = kpre[c];
            klb = lpre[c];
          }
        if (inbox) {
          ok = key >= 0 && (key >> 16) == m;
          if (ok) {
            const double thr = (double)klb - bx[7];
            const int sk = key & 0xFFFF;
            if (sk >= 0xFFF0) {
              ok = thr > ca.r_cut;
              side = sk == 0xFFFE ? 1 : 0;
            } else {
              // the kept segment and COUP_WIN on each side (lowest index on
              // equal distances, whatever the order), walked along the ring;
              // each vertex is loaded two segments before it is needed, so
              // the loads of three vertices are in flight at once
              constexpr int NW = 2 * COUP_WIN + 2;  // vertices of the window
              auto nxt = [&](int v) { return (v + 1 == n) ? 0 : v + 1; };
              int q = (sk - COUP_WIN) % n;
              if (q < 0) q += n;
              int q1 = nxt(q), q2 = nxt(q1);
              double ax = X[3 * q], ay = X[3 * q + 1];
              double b1x = X[3 * q1], b1y = X[3 * q1 + 1];
              double b2x = X[3 * q2], b2y = X[3 * q2 + 1];
#pragma unroll
              for (int k = 0; k + 1 < NW; k++) {
                // vertex k + 3 (the last ones load their predecessor again)
                const int q3 = k + 3 < NW ? nxt(q2) : q2;
                const double b3x = X[3 * q3], b3y = X[3 * q3 + 1];
                double tt;
                const double d2 = seg_d2(px, py, ax, ay, b1x, b1y, tt);
                if (d2 < d2b || (d2 == d2b && q < sb)) {
                  d2b = d2;
                  sb = q;
                  tb = tt;
                }
                q = q1;
                q1 = q2;
                q2 = q3;
                ax = b1x;
                ay = b1y;
                b1x = b2x;
                b1y = b2y;
                b2x = b3x;
                b2y = b3y;
              }
              ok = sqrt(d2b) < thr;
            }
          }
        }
        // Entries that have expired are renewed node by node, up to
        // COUP_RENEW per wave: the node's wave searches the whole ring for
        // it (FP32 screening relative to the box centre, FP64 for every
        // segment within the screening tolerance of the FP32 minimum, lowest
        // index on ties) and keeps either its closest segment with the exact
        // bound over all segments beyond the window, or, well beyond the
        // band, its side and distance.
        const bool renew = !ok && inbox && key >= 0 && (key >> 16) == m;
        unsigned long long need = __ballot(renew);
        if (__popcll(need) > COUP_RENEW) need = 0;  // left to the full search
        if (need) {
          const float4* stab = md.stab + b;
          const float* sinv = md.sinv + b;
          while (need) {
            const int ln = __ffsll((long long)need) - 1;
            need &= need - 1;
            const double qx = __shfl(px, ln, 64), qy = __shfl(py, ln, 64);
            const float fcx = (float)(qx - cx), fcy = (float)(qy - cy);
            float bf = 3.0e38f;
            for (int l = lane; l < n; l += 64) bf = fminf(bf, seg_d2f(fcx, fcy, stab[l], sinv[l]));
            bf = wave_minf(bf);
            const float tol = 2e-3f + 2e-5f * bf;
            double rd2 = 1e300, rt = 0.0;
            int rs = 0x7fffffff;
            for (int l = lane; l < n; l += 64) {
              if (seg_d2f(fcx, fcy, stab[l], sinv[l]) > bf + tol) continue;
              const int l1 = (l + 1 == n) ? 0 : l + 1;
              double tt;
              const double d2 = seg_d2(qx, qy, X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1], tt);
              if (d2 < rd2 || (d2 == rd2 && l < rs)) {
                rd2 = d2;
                rs = l;
                rt = tt;
              }
            }
            for (int o2 = 32; o2 > 0; o2 >>= 1) {
              const double d2o = __shfl_xor(rd2, o2, 64), to = __shfl_xor(rt, o2, 64);
              const int so = __shfl_xor(rs, o2, 64);
              if (d2o < rd2 || (d2o == rd2 && so < rs)) {
                rd2 = d2o;
                rs = so;
                rt = to;
              }
            }
            float o2m = 3.0e38f;
            for (int l = lane; l < n; l += 64) {
              int dd = abs(l - rs);
              dd = min(dd, n - dd);
              if (dd > COUP_WIN) o2m = fminf(o2m, seg_d2f(fcx, fcy, stab[l], sinv[l]));
            }
            o2m = wave_minf(o2m);
            if (lane == ln) {
              d2b = rd2;
              sb = rs;
              tb = rt;
              side = -1;
              const double d = sqrt(rd2);
              if (d > ca.r_cut + COUP_BEYOND) {
                const bool in = ring_side(X, n, o, sb, tb, px, py);
                ca.ckey[cix] = (m << 16) | (in ? 0xFFFE : 0xFFFD);
                ca.clb[cix] = __double2float_rd(d - 1e-3 - 1e-5 * d + bx[7]);
              } else {
                const double lb = sqrt(fmax((double)o2m - (2e-3 + 2e-5 * (double)o2m), 0.0));
                ca.ckey[cix] = (m << 16) | sb;
                ca.clb[cix] = __double2float_rd(lb - 1e-3 - 1e-5 * lb + bx[7]);
              }
              ok = true;
            }
          }
        }
        cached = __syncthreads_and(ok) != 0;
        if (!cached) {
          d2b = 1e300;
          tb = 0.0;
          sb = -1;
          side = -1;
        }
      }
      // lower bound to keep for this node after a full search (in the form
      // stored: less the drift) and its key; -1: nothing kept
      int keyw = -1;
      double lbw = 0.0;
      if (!cached) {
      // distance of the tile centre to the ring, in FP32 from the step's
      // segment table (the first values stay in registers for the
      // candidate list); the ray parity only for a tile beyond the band
      const float4* stab = md.stab + b;
      const float* sinv = md.sinv + b;
      const float pcx = (float)(pxt - cx), pcy = (float)(pyt - cy);
      constexpr int KEEPD = COUP_CHUNK / NT;
      float dl = 3.0e38f, dkeep[KEEPD];
#pragma unroll
      for (int r = 0; r < KEEPD; r++) {
        const int l = threadIdx.x + r * NT;
        dkeep[r] = l < n ? seg_d2f(pcx, pcy, stab[l], sinv[l]) : 3.0e38f;
        dl = fminf(dl, dkeep[r]);
      }
      for (int l = threadIdx.x + KEEPD * NT; l < n; l += NT) dl = fminf(dl, seg_d2f(pcx, pcy, stab[l], sinv[l]));
      const float dminf = sqrtf(block_minf<NT>(dl, s_redf));
      if ((double)dminf > ca.r_cut + rn16 + 0.01 + (cslot ? COUP_BEYOND : 0.0f)) {
        // no node of the tile is within the band: all on the centre's side
        int cr = 0;
        for (int l = threadIdx.x; l < n; l += NT) {
          const int l1 = (l + 1 == n) ? 0 : l + 1;
          cr += ray_cross(pxt, pyt, X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1]);
        }
        const int par = ((int)block_sum<NT>((double)cr, s_red)) & 1;
        if (inbox) Itot += par ? 1.0 : 0.0;
        if (slot < COUP_KEEP) b_seg[slot][threadIdx.x] = -1;
        if (cslot && valid) {
          // every node is at least dmin - rn16 from the ring
          // (outside the grown box: farther than reach, on the outside)
          ca.ckey[cix] = (m << 16) | (inbox && par ? 0xFFFE : 0xFFFD);
          ca.clb[cix] = __double2float_rd((inbox ? (double)dminf - rn16 - 0.011 : reach - 1e-3) + bx[7]);
        }
        continue;
      }
      // every node's closest segment lies within dmin + 2 rn16 of the
      // centre.  Candidates go to LDS with their geometry relative to the
      // tile centre in FP32 and their end points in FP64; each node finds
      // the FP32 minimum, then re-evaluates in FP64 every candidate within a
      // margin that covers the FP32 rounding, so the FP64 closest segment
      // (lowest index on ties) is the one chosen.
      const float pad = cslot ? COUP_PAD : 0.0f;
      const float cull = dminf + (float)(2.0 * rn16) + 0.01f + pad;
      const float fx = (float)(px - pxt), fy = (float)(py - pyt);
      for (int c0 = 0; c0 < n; c0 += COUP_CHUNK) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        for (int l = c0 + threadIdx.x; l < min(n, c0 + COUP_CHUNK); l += NT) {
          const int r = (l - threadIdx.x) / NT;
          const float d = (c0 == 0 && r < KEEPD) ? dkeep[r] : seg_d2f(pcx, pcy, stab[l], sinv[l]);
          if (d <= cull * cull) {
            const int q = atomicAdd(&s_cnt, 1);
            const float4 sg = stab[l];
            const int l1 = (l + 1 == n) ? 0 : l + 1;
            s_cand[q] = l;
            s_geo[q] = make_float4(sg.x - pcx, sg.y - pcy, sg.z, sg.w);
            s_inv[q] = sinv[l];
            s_end[q] = make_double4(X[3 * l], X[3 * l + 1], X[3 * l1], X[3 * l1 + 1]);
          }
        }
        __syncthreads();
        const int nc = s_cnt;
        if (n <= COUP_CHUNK) {
          // one chunk holds every candidate: each wave narrows the list to
          // its 8 x 8 sub-tile (closest segments of its nodes lie within
          // d(sub-tile centre) + 2 rn8 of the sub-tile centre)
          auto d2f = [&](int q, float px_, float py_) {
            const float4 g4 = s_geo[q];
            const float qx = px_ - g4.x, qy = py_ - g4.y;
            const float sp = fminf(fmaxf((qx * g4.z + qy * g4.w) * s_inv[q], 0.0f), 1.0f);
            const float dx = qx - sp * g4.z, dy = qy - sp * g4.w;
            return dx * dx + dy * dy;
          };
          float dw = 3.0e38f;
          for (int q = lane; q < nc; q += 64) dw = fminf(dw, d2f(q, cwx, cwy));
          for (int o2 = 32; o2 > 0; o2 >>= 1) dw = fminf(dw, __shfl_xor(dw, o2, 64));
          const float cr = sqrtf(dw) + (float)(2.0 * rn8) + 1e-3f + pad;
          int cnt = 0;
          for (int base = 0; base < nc; base += 64) {
            const int q = base + lane;
            const bool pr = q < nc && d2f(q, cwx, cwy) <= cr * cr;
            const unsigned long long mk = __ballot(pr);
            if (pr) s_wl[wv][cnt + __popcll(mk & below)] = (unsigned short)q;
            cnt += __popcll(mk);
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
          // side of the sub-tile centre, from its exact closest segment
          auto centre_side = [&]() {
            double d2c, tc;
            int sc;
            wave_closest(s_wl[wv], cnt, s_cand, s_geo, s_inv, s_end, cwx, cwy, dw, pxt + cwx, pyt + cwy, d2c, sc,
                         tc);
            return ring_side(X, n, o, sc, tc, pxt + cwx, pyt + cwy) ? 1 : 0;
          };
          const float rb = (float)(ca.r_cut + rn8) + (cslot ? COUP_BEYOND : 0.0f);
          // segments off this wave's list lie farther than cr from the
          // sub-tile centre (and those off the tile's list farther than
          // cull - 4 sqrt 2): at least lout from any node of the sub-tile
          const double lout = fmin((double)cr, (double)cull - 4.0 * 1.41421356237309515) - rn8;
          if (shortcut && dw - (2e-3f + 2e-5f * dw) > rb * rb) {
            // the whole sub-tile lies beyond the band
            side = centre_side();
            if (inbox) {
              keyw = (m << 16) | (side ? 0xFFFE : 0xFFFD);
              lbw = fmin(sqrt(fmax((double)dw - (2e-3 + 2e-5 * (double)dw), 0.0)),
                         (double)cull - 4.0 * 1.41421356237309515) - rn8;
            }
          } else {
            float bf = 3.0e38f;
            if (inbox)
              for (int k = 0; k < cnt; k++) bf = fminf(bf, d2f(s_wl[wv][k], fx, fy));
            const float tol = 2e-3f + 2e-5f * bf;
            const float rc = (float)ca.r_cut;
            const bool beyond = shortcut && !cslot && inbox && bf - tol > rc * rc;
            if (__ballot(beyond)) {
              const int sc = centre_side();
              if (beyond) side = sc;
            }
            if (beyond) {
              keyw = (m << 16) | (side ? 0xFFFE : 0xFFFD);
              lbw = fmin(sqrt(fmax((double)bf - (double)tol, 0.0)), lout);
            }
            if (inbox && !beyond) {
              for (int k = 0; k < cnt; k++) {
                const int q = s_wl[wv][k];
                if (d2f(q, fx, fy) > bf + tol) continue;
                const int s = s_cand[q];
                const double4 e = s_end[q];
                double tt;
                const double d2 = seg_d2(px, py, e.x, e.y, e.z, e.w, tt);
                if (d2 < d2b || (d2 == d2b && s < sb)) {
                  d2b = d2;
                  sb = s;
                  tb = tt;
                }
              }
              if (cslot && sb >= 0) {
                // nearest listed segment more than COUP_WIN from sb
                float o2 = 3.0e38f;
                for (int k = 0; k < cnt; k++) {
                  const int q = s_wl[wv][k];
                  int dd = abs(s_cand[q] - sb);
                  dd = min(dd, n - dd);
                  if (dd <= COUP_WIN) continue;
                  o2 = fminf(o2, d2f(q, fx, fy));
                }
                keyw = (m << 16) | sb;
                lbw = fmin(sqrt(fmax((double)o2 - (2e-3 + 2e-5 * (double)o2), 0.0)), lout);
              }
            }
          }
        } else if (inbox && nc > 0) {
          float bf = 3.0e38f;
          for (int q = 0; q < nc; q++) {
            const float4 g4 = s_geo[q];
            const float qx = fx - g4.x, qy = fy - g4.y;
            const float sp = fminf(fmaxf((qx * g4.z + qy * g4.w) * s_inv[q], 0.0f), 1.0f);
            const float dx = qx - sp * g4.z, dy = qy - sp * g4.w;
            bf = fminf(bf, dx * dx + dy * dy);
          }
          const float tol = 2e-3f + 2e-5f * bf;
          for (int q = 0; q < nc; q++) {
            const float4 g4 = s_geo[q];
            const float qx = fx - g4.x, qy = fy - g4.y;
            const float sp = fminf(fmaxf((qx * g4.z + qy * g4.w) * s_inv[q], 0.0f), 1.0f);
            const float dx = qx - sp * g4.z, dy = qy - sp * g4.w;
            if (dx * dx + dy * dy > bf + tol) continue;
            const int s = s_cand[q];
            const double4 e = s_end[q];
            double tt;
            const double d2 = seg_d2(px, py, e.x, e.y, e.z, e.w, tt);
            if (d2 < d2b || (d2 == d2b && s < sb)) {
              d2b = d2;
              sb = s;
              tb = tt;
            }
          }
        }
        __syncthreads();
      }
      if (cslot && valid && !inbox) {
        // outside the box grown by reach: farther than reach from the ring
        keyw = (m << 16) | 0xFFFD;
        lbw = reach;
      }
      if (cslot && keyw >= 0 && (keyw & 0xFFFF) < 0xFFF0 && sqrt(d2b) > ca.r_cut + COUP_BEYOND) {
        // well beyond the band: keep the side and the distance instead (a
        // node near the ring's medial axis has no room between its closest
        // segments)
        keyw = (m << 16) | (ring_side(X, n, o, sb, tb, px, py) ? 0xFFFE : 0xFFFD);
        lbw = sqrt(d2b);
      }
      if (cslot && valid) {
        // FP32 distances are within 1e-5 of exact here: a margin of 1e-3
        // plus 1e-5 of the bound; stored with the drift so far added and
        // rounded down, so the bound at a later step is the stored value
        // less the drift then
        ca.ckey[cix] = keyw;
        ca.clb[cix] = keyw >= 0 ? __double2float_rd(lbw - 1e-3 - 1e-5 * fabs(lbw) + bx[7]) : 0.0f;
      }
      }  // !cached
      bool band = false;
      double gx = 0.0, gy = 0.0;
      if (inbox && side >= 0) {
        Itot += side ? 1.0 : 0.0;
      } else if (inbox && sb >= 0) {
        const double d = sqrt(d2b);
        const int sb1 = (sb + 1 == n) ? 0 : sb + 1;
        const double eax = X[3 * sb], eay = X[3 * sb + 1], ebx = X[3 * sb1], eby = X[3 * sb1 + 1];
        const bool in = ring_side_ab(X, n, o, sb, tb, eax, eay, ebx, eby, px, py);
        const double sd = in ? d : -d;
        band = d <= ca.r_cut;
        if (band) {
          double s2;
          Itot += profile_sech2(sd / (2.0 * ca.alpha), s2);
          if (ca.want_force) band_push(eax, eay, ebx, eby, tb, px, py, sd, s2, gx, gy);
        } else {
          Itot += in ? 1.0 : 0.0;
        }
      }
      if (slot < COUP_KEEP) {
        b_seg[slot][threadIdx.x] = band ? sb : -1;
        b_t[slot][threadIdx.x] = tb;
        b_gx[slot][threadIdx.x] = gx;
        b_gy[slot][threadIdx.x] = gy;
      }
    }
    if (valid) Ifield[node] = Itot;
    if (ca.want_force) {
      // coupling force on the markers, -dE_c/dX (eq. DiscreteCF): from every
      // band node, kappa_c/(4 alpha) (psi - I) sech^2(d/2 alpha) dd/dX_v with
      // dd/dX_v = -sign(d) nhat w_v (nhat from the closest point to the
      // node, w_v the closest point's weight on vertex v)
      if (nm > COUP_KEEP && threadIdx.x == 0) md.status[1] = 1;
      const int nk = min(nm, COUP_KEEP);
      bool anyband = false;
      for (int slot = 0; slot < nk; slot++) anyband |= b_seg[slot][threadIdx.x] >= 0;
      // psi only where a node of the wave is in a band
      double psi = 0.0;
      if (valid && __ballot(anyband)) {
        psi = hrest;
#pragma unroll
        for (int i = 0; i < 8; i++) psi += (double)hmov[i];
      }
      // per membrane: the tile's contributions are summed in LDS (integer
      // adds of fixed-point values, so the order does not matter), indexed
      // around the closest segment of one of its band nodes, then added to
      // the markers with one global atomic each; a marker out of the LDS
      // window is added directly
      for (int slot = 0; slot < nk; slot++) {
        const int b = s_mof[slot][0], n = s_mof[slot][1] - b;
        const int sb = b_seg[slot][threadIdx.x];
        const double tb = b_t[slot][threadIdx.x];
        const double ux = b_gx[slot][threadIdx.x], uy = b_gy[slot][threadIdx.x];
        const bool live = sb >= 0 && (ux != 0.0 || uy != 0.0);
        if (threadIdx.x == 0) s_base = -1;
        for (int i = threadIdx.x; i < COUP_FACC; i += NT) s_facc[i][0] = s_facc[i][1] = 0;
        __syncthreads();
        if (live) atomicCAS(&s_base, -1, sb);
        __syncthreads();
        const int base = s_base;
        if (base < 0) continue;  // no band node of this membrane in the tile (uniform)
        if (live) {
          const int s1 = (sb + 1 == n) ? 0 : sb + 1;
          const double wgt = ca.kappa_c / (4.0 * ca.alpha) * (psi - Itot);
          const double gx = ux * wgt, gy = uy * wgt;
          const int vv[2] = {sb, s1};
          const double ww[2] = {1.0 - tb, tb};
#pragma unroll
          for (int e = 0; e < 2; e++) {
            int dd = vv[e] - base;
            if (dd > n / 2) dd -= n;
            if (dd < -(n / 2)) dd += n;
            const int la = dd + COUP_FACC / 2;
            const long long vx = to_fix(gx * ww[e]), vy = to_fix(gy * ww[e]);
            if (la >= 0 && la < COUP_FACC) {
              atomicAdd((unsigned long long*)&s_facc[la][0], (unsigned long long)vx);
              atomicAdd((unsigned long long*)&s_facc[la][1], (unsigned long long)vy);
            } else {
              long long* A = md.Facc + 3 * (b + vv[e]);
              atomicAdd((unsigned long long*)&A[0], (unsigned long long)vx);
              atomicAdd((unsigned long long*)&A[1], (unsigned long long)vy);
            }
          }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < COUP_FACC; i += NT) {
          const long long vx = s_facc[i][0], vy = s_facc[i][1];
          if (vx == 0 && vy == 0) continue;
          const int v = ((base + i - COUP_FACC / 2) % n + n) % n;
          long long* A = md.Facc + 3 * (b + v);
          atomicAdd((unsigned long long*)&A[0], (unsigned long long)vx);
          atomicAdd((unsigned long long*)&A[1], (unsigned long long)vy);
        }
        __syncthreads();
      }
    }
    __syncthreads();  // LDS band data and lists are rewritten by the next tile
  }
}

// one tile per workgroup (grid-stride over the active-tile list)
template <class St, typename R, int NT>
// (the LDS of a workgroup leaves room for two per CU: registers are sized
// for two waves per SIMD)
__global__ __launch_bounds__(NT, 2) void k_coupling2d(MemDev md, TileMap tm, CoupArgs ca,
                                                   double* __restrict__ Ifield, St cur,
                                                   const int* __restrict__ cnt) {
  const int ntl = *cnt;  // active tiles (the counter the tile pass used)
  for (int li = blockIdx.x; li < ntl; li += gridDim.x) coupling2d_tile<St, R, NT>(md, tm, ca, Ifield, cur, li);
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

// Strain energy W per unit rest length of a ring segment stretched by lam
// and its tension dW/dlam.  0: eq. DiscreteSE, ks/2 (lam - 1)^2.  1 and 2:
// the neo-Hookean and Skalak membrane laws with the second principal stretch
// held at 1 (plane strain, of which a 2D ring is the section), with moduli
// giving the same small-strain stiffness ks: ks/8 (lam - 1/lam)^2 and
// ks/8 (lam^2 - 1)^2.
__device__ __forceinline__ double seg_tension(int law, double ks, double lam) {
  if (law == 1) return 0.25 * ks * (lam - 1.0 / lam) * (1.0 + 1.0 / (lam * lam));
  if (law == 2) return 0.5 * ks * lam * (lam * lam - 1.0);
  return ks * (lam - 1.0);
}
__device__ __forceinline__ double seg_energy(int law, double ks, double lam) {
  if (law == 1) {
    const double q = lam - 1.0 / lam;
    return 0.125 * ks * q * q;
  }
  if (law == 2) {
    const double q = lam * lam - 1.0;
    return 0.125 * ks * q * q;
  }
  const double q = lam - 1.0;
  return 0.5 * ks * q * q;
}

// one term of marker g's force (eq. DiscreteTF), by lane k of its group:
// k = 0, 1 the strain of segments l -> l+1 and l-1 -> l (eq. DiscreteSF,
// each pulling with its tension along itself), k = 2, 3, 4 the bending terms
// of vertices l-1, l, l+1, which depend on X_l (eq. DiscreteBF), k = 5 the
// coupling force accumulated by the profile kernel (read and cleared).
// Returns the membrane's bending modulus.
__device__ __forceinline__ double memforce2d_part(const MemDev& md, int g, int k, double& tx, double& ty) {
  const int m = md.mid[g];
  const int b = md.moff[m], n = md.moff[m + 1] - b;
  const int l = g - b;
  const double kbm = md.kb[m];
  tx = ty = 0.0;
  // marker l + j for |j| <= 2 (a ring holds at least three markers)
  auto at = [&](int j) {
    int i = l + j;
    if (i < 0) i += n;
    if (i >= n) i -= n;
    return b + i;
  };
  if (k <= 1) {
    const int v = at(-k), w = at(1 - k);
    const double ex = md.X[3 * w] - md.X[3 * v], ey = md.X[3 * w + 1] - md.X[3 * v + 1];
    const double len = sqrt(ex * ex + ey * ey);
    const double s = seg_tension(md.law[m], md.ks[m], len / md.rest[v]) / len;
    // X_l is the start of segment l -> l+1 and the end of l-1 -> l
    tx = k == 0 ? s * ex : -(s * ex);
    ty = k == 0 ? s * ey : -(s * ey);
  } else if (k <= 4) {
    if (kbm != 0.0) {
      // vertex v = l + k - 3: a = X_{v+1} - X_v, b = X_v - X_{v-1}
      const int u = at(k - 4), v = at(k - 3), w = at(k - 2);
      double gax, gay, gbx, gby, e;
      bend_grad(md.X[3 * w] - md.X[3 * v], md.X[3 * w + 1] - md.X[3 * v + 1], md.X[3 * v] - md.X[3 * u],
                md.X[3 * v + 1] - md.X[3 * u + 1], kbm, gax, gay, gbx, gby, e);
      // X_l enters vertex l-1 through a (+1), vertex l through a (-1) and b
      // (+1), vertex l+1 through b (-1)
      if (k == 2) {
        tx = -gax;
        ty = -gay;
      } else if (k == 3) {
        tx = gax - gbx;
        ty = gay - gby;
      } else {
        tx = gbx;
        ty = gby;
      }
    }
  } else if (k == 5) {
    long long* acc = md.Facc + 3 * g;
    tx = from_fix(acc[0]);
    ty = from_fix(acc[1]);
    acc[0] = 0;
    acc[1] = 0;
    acc[2] = 0;
  }
  return kbm;
}

// spreading, eq. Spreading with delta x = 1 (READING: no extra Delta s):
// sixteen lanes per marker, each adds F delta_h(x - X) to one stencil node in
// fixed point (integer sums are order independent)
__device__ __forceinline__ void spread2d_run(const MemDev& md, long long* __restrict__ fib, int nx, int ny,
                                             int wall_y, int g, int k, double Fx, double Fy) {
  const double X = md.X[3 * g], Y = md.X[3 * g + 1];
  const int cx = (int)floor(X) - 1 + (k & 3), cy = (int)floor(Y) - 1 + (k >> 2);
  if (wall_y && (cy < 0 || cy >= ny)) return;
  const double w = peskin(cx - X) * peskin(cy - Y);
  const long long node = (long long)wrap(cy, ny) * nx + wrap(cx, nx);
  atomicAdd((unsigned long long*)&fib[2 * node], (unsigned long long)to_fix(Fx * w));
  atomicAdd((unsigned long long*)&fib[2 * node + 1], (unsigned long long)to_fix(Fy * w));
}

// marker forces (strain + bending + coupling, eq. DiscreteTF): six lanes of
// each sixteen-lane group form one term each, the group sums them by
// shuffles, then all sixteen spread; every lane of a group must call it
__device__ __forceinline__ void forcespread2d_run(const MemDev& md, long long* __restrict__ fib, int nx, int ny,
                                                  int wall_y, int g, int k, bool live) {
  double tx = 0.0, ty = 0.0, kbm = 0.0;
  if (live && k < 6) kbm = memforce2d_part(md, g, k, tx, ty);
  kbm = __shfl(kbm, 0, 16);
  // the terms added in a fixed order: strain, bending (when the membrane has
  // a bending modulus), coupling
  double Fx = __shfl(tx, 0, 16), Fy = __shfl(ty, 0, 16);
  Fx += __shfl(tx, 1, 16);
  Fy += __shfl(ty, 1, 16);
#pragma unroll
  for (int j = 2; j < 5; j++) {
    const double bx = __shfl(tx, j, 16), by = __shfl(ty, j, 16);
    if (kbm != 0.0) {
      Fx += bx;
      Fy += by;
    }
  }
  Fx += __shfl(tx, 5, 16);
  Fy += __shfl(ty, 5, 16);
  if (live && k == 0) {
    if (!(fabs(Fx) < FIX_LIMIT) || !(fabs(Fy) < FIX_LIMIT)) md.status[0] = 1;
    md.F[3 * g] = Fx;
    md.F[3 * g + 1] = Fy;
    md.F[3 * g + 2] = 0.0;
  }
  if (live) spread2d_run(md, fib, nx, ny, wall_y, g, k, Fx, Fy);
}

__global__ void k_forcespread2d(MemDev md, long long* __restrict__ fib, int nx, int ny, int wall_y) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = tid >> 4, k = tid & 15;
  forcespread2d_run(md, fib, nx, ny, wall_y, g, k, g < md.M);
}

// interpolation of v* = u(t+1) + f(t) / (2 rho(t+1)) at the stencil of X(t)
// (eq. Interpolation, READING: the force of step t stands in for the unknown
// force at t+1), then X(t+1) = X(t) + U (eq. UpdatedXl).  Sixteen lanes per
// marker (one stencil node each), summed in a fixed butterfly order.
// all sixteen lanes of a marker group must call it (live false for padding)
template <class St, typename R>
__device__ __forceinline__ void interp2d_run(const MemDev& md, const St& cur, const LBParams& P,
                                             const double* __restrict__ force, int g, int k, bool live) {
  using L = Lattice<9>;
  double Ux = 0, Uy = 0;
  double X = 0, Y = 0;
  if (live) {
    X = md.X[3 * g];
    Y = md.X[3 * g + 1];
    const int cx = (int)floor(X) - 1 + (k & 3), cy = (int)floor(Y) - 1 + (k >> 2);
    if (!(P.wall_y && (cy < 0 || cy >= P.ny))) {
      const int yw = wrap(cy, P.ny), xw = wrap(cx, P.nx);
      const long long node = (long long)yw * P.nx + xw;
      // neighbour rows and columns of the stencil node, wrapped once
      const long long rlo = (long long)(yw == 0 ? P.ny - 1 : yw - 1) * P.nx;
      const long long rhi = (long long)(yw == P.ny - 1 ? 0 : yw + 1) * P.nx;
      const int xlo = xw == 0 ? P.nx - 1 : xw - 1, xhi = xw == P.nx - 1 ? 0 : xw + 1;
      const bool wlo = P.wall_y && yw == 0, whi = P.wall_y && yw == P.ny - 1;
      double d = 0, jx = 0, jy = 0;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        const bool back = L::cy[i] > 0 ? wlo : (L::cy[i] < 0 ? whi : false);
        const long long row = L::cy[i] > 0 ? rlo : (L::cy[i] < 0 ? rhi : node - xw);
        const int col = L::cx[i] > 0 ? xlo : (L::cx[i] < 0 ? xhi : xw);
        const double v = (double)cur.template load<R>(0, back ? L::opp[i] : i, back ? node : row + col);
        d += v;
        jx += L::cx[i] * v;
        jy += L::cy[i] * v;
      }
      const double rho = P.rho0 + d;
      const double w = peskin(cx - X) * peskin(cy - Y);
      Ux = w * (jx + 0.5 * force[2 * node]) / rho;
      Uy = w * (jy + 0.5 * force[2 * node + 1]) / rho;
    }
  }
  for (int o = 8; o > 0; o >>= 1) {
    Ux += __shfl_xor(Ux, o, 16);
    Uy += __shfl_xor(Uy, o, 16);
  }
  if (live && k == 0) {
    md.U[3 * g] = Ux;
    md.U[3 * g + 1] = Uy;
    md.U[3 * g + 2] = 0.0;
    md.X[3 * g] = X + Ux;
    md.X[3 * g + 1] = Y + Uy;

  }
}

template <class St, typename R>
__global__ void k_interp2d(MemDev md, St cur, LBParams P, const double* __restrict__ force) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = tid >> 4, k = tid & 15;
  interp2d_run<St, R>(md, cur, P, force, g, k, g < md.M);
}

}  // namespace lb
