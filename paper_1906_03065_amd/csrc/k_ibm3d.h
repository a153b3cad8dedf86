// k_ibm3d.h -- membrane side of the step for closed triangle meshes (D3Q19):
// face and vertex normals, coupling profile and coupling force (eqs. Iprofile,
// DiscreteCE, DiscreteCF with d the signed distance to the mesh), edge-spring
// and dihedral forces (the 3D membrane law of this library: edge springs
// kappa_s/2 sum (l/l0 - 1)^2 l0 and bending kappa_b sum_e (1 - cos theta_e)),
// spreading and interpolation with the tensor-product four-point kernel
// (eqs. Spreading, DiscreteDirac, Interpolation, UpdatedXl).  FP64 throughout.
//
// Sign of d: the closest point of the closest triangle lies in its interior,
// on an edge or at a vertex; the side is taken against the face normal, the
// sum of the two face normals of the edge, or the angle-weighted vertex
// normal (exact for a closed, non-self-intersecting mesh).
#pragma once
#include "common.h"
#include "k_ibm.h"
#include "k_lb.h"
#include "k_lb3d.h"

namespace lb {

constexpr int TILE3 = 8;
constexpr int COUP3_THREADS = 512;  // one thread per node of an 8^3 tile
constexpr int COUP3_KEEP = 2;
// the coupling forces of a tile's band nodes are summed per marker in an LDS
// hash table of this many markers (open addressing) before one global
// atomic per marker and component; a marker that finds the table full adds
// straight to global memory
constexpr int COUP3_HASH = 512;
// Temporal coherence (as in 2D): each node keeps, for up to COUP3_CACHE
// membranes of its tile, either its closest triangle t with a lower bound
// on the distance of every triangle that shares no vertex with t, or (beyond
// the band) its side and a lower bound on its distance.  With the cache on
// the candidate lists reach COUP3_PAD farther and a tile or sub-tile is
// taken to lie beyond the band without a node search only COUP3_BEYOND
// farther out, so that entries outlast some drift of the markers.
constexpr int COUP3_CACHE = 2;
constexpr float COUP3_PAD = 2.0f;
constexpr float COUP3_BEYOND = 1.0f;
constexpr int C3_KEYB = 20;         // key = membrane << 20 | triangle (or a beyond code)
constexpr int C3_IN = 0xFFFFE, C3_OUT = 0xFFFFD;

struct MeshDev {
  int* tri;       // 3 per triangle, marker ids
  int* toff;      // K+1 triangle offsets
  int* edge;      // 4 per edge: a, b, t1, t2
  double* erest;  // rest length per edge
  int* eoff;      // K+1 edge offsets
  int* tadj;      // 3 per triangle: the triangle across edge (v_k, v_k+1)
  int* tedge;     // 3 per triangle: the edge opposite vertex k
  int* vtoff;     // M+1: vertex -> incident triangles (CSR)
  int* vt;
  double* fn;     // 3 per triangle: unit face normal (area vector direction)
  double* vn;     // 3 per vertex: angle-weighted normal
  int* coff;      // K+1 offsets of the 64-triangle clusters of each mesh
  int T, E;
};

__device__ __forceinline__ void sub3(const double* a, const double* b, double* c) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}
__device__ __forceinline__ double dot3d(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3d(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
__global__ void k_facenormals(MemDev md, MeshDev mh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mh.T) return;
  const double* p0 = md.X + 3 * mh.tri[3 * t];
  const double* p1 = md.X + 3 * mh.tri[3 * t + 1];
  const double* p2 = md.X + 3 * mh.tri[3 * t + 2];
  double e1[3], e2[3], n[3];
  sub3(p1, p0, e1);
  sub3(p2, p0, e2);
  cross3d(e1, e2, n);
  const double l = sqrt(dot3d(n, n));
  for (int a = 0; a < 3; a++) mh.fn[3 * t + a] = l > 0 ? n[a] / l : 0.0;
}

// angle-weighted pseudo-normal of every vertex (sum over incident faces of
// the face angle at the vertex times the unit face normal)
__global__ void k_vertexnormals(MemDev md, MeshDev mh) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= md.M) return;
  double n[3] = {0, 0, 0};
  for (int q = mh.vtoff[v]; q < mh.vtoff[v + 1]; q++) {
    const int t = mh.vt[q];
    int k = 0;
    while (k < 3 && mh.tri[3 * t + k] != v) k++;
    const double* pv = md.X + 3 * v;
    const double* pa = md.X + 3 * mh.tri[3 * t + (k + 1) % 3];
    const double* pb = md.X + 3 * mh.tri[3 * t + (k + 2) % 3];
    double ea[3], eb[3];
    sub3(pa, pv, ea);
    sub3(pb, pv, eb);
    const double c = dot3d(ea, eb) / sqrt(dot3d(ea, ea) * dot3d(eb, eb));
    const double ang = acos(fmin(1.0, fmax(-1.0, c)));
    for (int a = 0; a < 3; a++) n[a] += ang * mh.fn[3 * t + a];
  }
  const double l = sqrt(dot3d(n, n));
  for (int a = 0; a < 3; a++) mh.vn[3 * v + a] = l > 0 ? n[a] / l : 0.0;
}

// orientation of each closed mesh from its signed volume (one block each)
template <int NT>
__global__ __launch_bounds__(NT) void k_meshvolume(MemDev md, MeshDev mh) {
  __shared__ double sh[NT / 64];
  const int m = blockIdx.x;
  double acc = 0.0;
  for (int t = mh.toff[m] + threadIdx.x; t < mh.toff[m + 1]; t += NT) {
    const double* p0 = md.X + 3 * mh.tri[3 * t];
    const double* p1 = md.X + 3 * mh.tri[3 * t + 1];
    const double* p2 = md.X + 3 * mh.tri[3 * t + 2];
    double c[3];
    cross3d(p1, p2, c);
    acc += dot3d(p0, c);
  }
  const double vol = block_sum<NT>(acc, sh);
  if (threadIdx.x == 0) md.mbox[8 * m + 6] = vol >= 0.0 ? 1.0 : -1.0;
}

// closest point of triangle (a, b, c) to p: squared distance, weights w of
// the closest point on a, b, c.  Projection onto the plane when it falls
// inside the triangle, otherwise the nearest of the three edges.
__device__ __forceinline__ double tri_d2(const double* p, const double* a, const double* b,
                                         const double* c, double* w) {
  double e0[3], e1[3], ap[3], n[3];
  sub3(b, a, e0);
  sub3(c, a, e1);
  sub3(p, a, ap);
  cross3d(e0, e1, n);
  const double nn = dot3d(n, n);
  if (nn > 0.0) {
    // barycentric coordinates of the projection: (u, v) on (b, c)
    double t0[3], t1[3];
    cross3d(ap, e1, t0);
    cross3d(e0, ap, t1);
    const double u = dot3d(t0, n) / nn, v = dot3d(t1, n) / nn;
    if (u > 0.0 && v > 0.0 && u + v < 1.0) {
      w[0] = 1.0 - u - v;
      w[1] = u;
      w[2] = v;
      const double h = dot3d(ap, n);
      return h * h / nn;
    }
  }
  // edges (a,b), (b,c), (c,a)
  const double* P[3] = {a, b, c};
  double best = 1e300;
  for (int k = 0; k < 3; k++) {
    const double* s0 = P[k];
    const double* s1 = P[(k + 1) % 3];
    double ed[3], sp[3];
    sub3(s1, s0, ed);
    sub3(p, s0, sp);
    const double ee = dot3d(ed, ed);
    double t = ee > 0.0 ? dot3d(sp, ed) / ee : 0.0;
    t = fmin(fmax(t, 0.0), 1.0);
    const double dx = sp[0] - t * ed[0], dy = sp[1] - t * ed[1], dz = sp[2] - t * ed[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < best) {
      best = d2;
      w[k] = 1.0 - t;
      w[(k + 1) % 3] = t;
      w[(k + 2) % 3] = 0.0;
    }
  }
  return best;
}

struct Coup3Args {
  int nx, ny, nz, wall_y, wall_z;
  double alpha, kappa_c, r_cut;
  int want_force;
  // per node and cached membrane slot (COUP3_CACHE x N): key and bound (plus
  // the membrane's drift when written); null disables the cache
  int* ckey;
  float* clb;
  long long N;
};

__device__ __forceinline__ double near_img(double v, double c, int n, int per) {
  return per ? v + n * floor((c - v) / n + 0.5) : v;
}

// Geometry of one tile against one membrane's box: images of the tile centre
// and of this thread's node nearest the box centre (the node image is the one
// the profile is defined with), whether the tile can be skipped, and whether
// its nodes fall into different periodic images (a tile that straddles the
// antipode of the box centre), in which case every node is searched alone.
struct TileGeo {
  double pc[3], pp[3];
  bool miss, split, inbox;
};

__device__ __forceinline__ TileGeo tile_geo(const double* bx, const double* ct, const int* xi,
                                            const int* t0, const int* dims, const int* per,
                                            double hd, double reach, bool valid) {
  TileGeo g;
  g.miss = false;
  g.split = false;
  g.inbox = valid;
  bool far = false;  // a split axis whose two runs of nodes both miss the grown box
  for (int a = 0; a < 3; a++) {
    const double cm = 0.5 * (bx[a] + bx[3 + a]);
    // the image of the tile's first node: the nodes of a tile that does not
    // split share one image, while a partial tile's nominal centre can lie
    // beyond the antipode
    g.pc[a] = ct[a] + (near_img((double)t0[a], cm, dims[a], per[a]) - t0[a]);
    g.pp[a] = near_img((double)xi[a], cm, dims[a], per[a]);
    const bool out = g.pc[a] + hd < bx[a] - reach || g.pc[a] - hd > bx[3 + a] + reach;
    if (g.pp[a] < bx[a] - reach || g.pp[a] > bx[3 + a] + reach) g.inbox = false;
    bool sa = false;
    if (per[a]) {
      const int s0 = t0[a], s1 = min(t0[a] + TILE3 - 1, dims[a] - 1);
      const double i0 = near_img((double)s0, cm, dims[a], 1), i1 = near_img((double)s1, cm, dims[a], 1);
      if (i0 - s0 != i1 - s1) {
        // the tile's nodes fall into two images (it straddles the antipode
        // of the box centre): the first image's nodes run from i0 up to the
        // antipode, the second image's from the antipode up to i1, and the
        // grown box, narrower than the period, reaches neither antipode side
        sa = true;
        far |= !(i0 <= bx[3 + a] + reach || i1 >= bx[a] - reach);
      }
    }
    g.split |= sa;
    if (!sa) g.miss |= out;
  }
  g.miss |= far;
  return g;
}

// ---------------------------------------------------------------------------
// Closest-triangle search.  Distances are first compared in FP32 (with
// margins far above the FP32 rounding), and every triangle whose FP32
// distance is within a tolerance of a point's FP32 minimum is re-evaluated
// in FP64, so the FP64 closest triangle (lowest index on exact ties) is the
// one chosen.  Levels: the whole mesh against the 8^3 tile centre (from a
// per-step FP32 table relative to the membrane's box centre), the tile's
// candidate list against the centre of each 4^3 sub-tile (one wave), and
// the sub-tile's list against each of its nodes.  At every level a bounding
// sphere per triangle gives |p - c| - r <= d(p, T) <= |p - c| + r: the least
// upper bound over the list caps the minimum, and only triangles whose lower
// bound reaches below it get the exact distance.

// per-step FP32 table: 4 float4 per triangle, relative to the box centre of
// the triangle's membrane: the vertices, then (centroid, bounding radius)
__global__ void k_tritable3d(MemDev md, MeshDev mh, float4* __restrict__ tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mh.T) return;
  int m = 0;
  while (m + 1 < md.K && mh.toff[m + 1] <= t) m++;
  const double* bx = md.mbox + 8 * m;
  const double c[3] = {0.5 * (bx[0] + bx[3]), 0.5 * (bx[1] + bx[4]), 0.5 * (bx[2] + bx[5])};
  const double* v[3];
  for (int k = 0; k < 3; k++) v[k] = md.X + 3 * mh.tri[3 * t + k];
  double g[3], r = 0.0;
  for (int a = 0; a < 3; a++) g[a] = (v[0][a] + v[1][a] + v[2][a]) / 3.0;
  for (int k = 0; k < 3; k++) {
    double d[3];
    sub3(v[k], g, d);
    r = fmax(r, sqrt(dot3d(d, d)));
    tab[4 * t + k] = make_float4((float)(v[k][0] - c[0]), (float)(v[k][1] - c[1]), (float)(v[k][2] - c[2]), 0.0f);
  }
  tab[4 * t + 3] = make_float4((float)(g[0] - c[0]), (float)(g[1] - c[1]), (float)(g[2] - c[2]),
                               (float)(r * (1.0 + 1e-6) + 1e-5));
}

// bounding sphere of every cluster of 64 consecutive triangles of a mesh,
// from the triangles' spheres (one wave per cluster)
constexpr int CL3 = 64;
__global__ void k_clusters3d(MemDev md, MeshDev mh, const float4* __restrict__ tab, float4* __restrict__ ctab,
                             int ncl) {
  const int gk = (int)((blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (gk >= ncl) return;
  int m = 0;
  while (m + 1 < md.K && mh.coff[m + 1] <= gk) m++;
  const int t0 = mh.toff[m] + (gk - mh.coff[m]) * CL3, t1 = min(t0 + CL3, mh.toff[m + 1]);
  const int t = t0 + lane;
  const bool live = t < t1;
  float4 sp = live ? tab[4 * t + 3] : make_float4(0.f, 0.f, 0.f, 0.f);
  float sx = sp.x, sy = sp.y, sz = sp.z;
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o, 64);
    sy += __shfl_xor(sy, o, 64);
    sz += __shfl_xor(sz, o, 64);
  }
  const float inv = 1.0f / (float)(t1 - t0);
  const float cx = sx * inv, cy = sy * inv, cz = sz * inv;
  float r = 0.0f;
  if (live) {
    const float dx = sp.x - cx, dy = sp.y - cy, dz = sp.z - cz;
    r = sqrtf(dx * dx + dy * dy + dz * dz) + sp.w;
  }
  for (int o = 32; o > 0; o >>= 1) r = fmaxf(r, __shfl_xor(r, o, 64));
  if (lane == 0) ctab[gk] = make_float4(cx, cy, cz, r * (1.0f + 1e-5f) + 1e-4f);
}

__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz) {
  return ax * bx + ay * by + az * bz;
}

// distance from p to the centre of bounding sphere s (radius in s.w)
__device__ __forceinline__ float sph_dist(float px, float py, float pz, float4 s) {
  const float dx = px - s.x, dy = py - s.y, dz = pz - s.z;
  return sqrtf(dx * dx + dy * dy + dz * dz);
}

// squared distance from p to the segment s0 + t e (t in [0,1]), ie = 1/|e|^2
__device__ __forceinline__ float seg_d2f(float px, float py, float pz, float ex, float ey, float ez,
                                         float ie) {
  const float t = fminf(fmaxf(dot3f(px, py, pz, ex, ey, ez) * ie, 0.0f), 1.0f);
  const float dx = px - t * ex, dy = py - t * ey, dz = pz - t * ez;
  return dx * dx + dy * dy + dz * dz;
}

// FP32 squared distance from p to triangle (a, b, c), all in one frame
__device__ __forceinline__ float tri_d2f_vtx(float px, float py, float pz, float4 a, float4 b, float4 c) {
  const float e0x = b.x - a.x, e0y = b.y - a.y, e0z = b.z - a.z;
  const float e1x = c.x - a.x, e1y = c.y - a.y, e1z = c.z - a.z;
  const float apx = px - a.x, apy = py - a.y, apz = pz - a.z;
  const float nx = e0y * e1z - e0z * e1y, ny = e0z * e1x - e0x * e1z, nz = e0x * e1y - e0y * e1x;
  const float nn = nx * nx + ny * ny + nz * nz;
  if (nn > 0.0f) {
    const float inn = 1.0f / nn;
    // u = ((ap x e1) . n) / nn, v = ((e0 x ap) . n) / nn
    const float u = ((apy * e1z - apz * e1y) * nx + (apz * e1x - apx * e1z) * ny + (apx * e1y - apy * e1x) * nz) * inn;
    const float v = ((e0y * apz - e0z * apy) * nx + (e0z * apx - e0x * apz) * ny + (e0x * apy - e0y * apx) * nz) * inn;
    if (u > 0.0f && v > 0.0f && u + v < 1.0f) {
      const float h = apx * nx + apy * ny + apz * nz;
      return h * h * inn;
    }
  }
  const float l0 = e0x * e0x + e0y * e0y + e0z * e0z, l1 = e1x * e1x + e1y * e1y + e1z * e1z;
  const float e2x = e1x - e0x, e2y = e1y - e0y, e2z = e1z - e0z;
  const float l2 = e2x * e2x + e2y * e2y + e2z * e2z;
  float d = seg_d2f(apx, apy, apz, e0x, e0y, e0z, l0 > 0.0f ? 1.0f / l0 : 0.0f);
  d = fminf(d, seg_d2f(apx, apy, apz, e1x, e1y, e1z, l1 > 0.0f ? 1.0f / l1 : 0.0f));
  d = fminf(d, seg_d2f(apx - e0x, apy - e0y, apz - e0z, e2x, e2y, e2z, l2 > 0.0f ? 1.0f / l2 : 0.0f));
  return d;
}

// candidate geometry in LDS, FP32 relative to the tile centre, precomputed in
// FP64: G0 = (a, 1/|e0|^2), G1 = (e0, 1/|e1|^2), G2 = (e1, 1/|e2|^2),
// G3 = (e1 x n)/|n|^2, G4 = (n x e0)/|n|^2, G5 = n/|n|, so that the
// barycentric coordinates of the projection are ap.G3, ap.G4; and the
// bounding sphere G6 = (centroid, radius)
constexpr int C3_LIST = 512;   // candidates whose geometry is staged at once
constexpr int C3_IDS = 4096;   // candidate ids of one tile
constexpr int C3_GEO = 7;
constexpr int C3_TIES = 8;    // near-ties a node keeps in registers

__device__ __forceinline__ void geo_store(float4 (*sg)[C3_LIST], int j, const double* a, const double* b,
                                          const double* c, const double* pc) {
  double e0[3], e1[3], e2[3], n[3], U[3], V[3], g[3];
  sub3(b, a, e0);
  sub3(c, a, e1);
  sub3(e1, e0, e2);
  cross3d(e0, e1, n);
  const double nn = dot3d(n, n);
  const double inn = nn > 0.0 ? 1.0 / nn : 0.0;
  cross3d(e1, n, U);
  cross3d(n, e0, V);
  const double l0 = dot3d(e0, e0), l1 = dot3d(e1, e1), l2 = dot3d(e2, e2);
  const double rn = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  for (int q = 0; q < 3; q++) g[q] = (a[q] + b[q] + c[q]) / 3.0;
  double r = 0.0;
  const double* P[3] = {a, b, c};
  for (int k = 0; k < 3; k++) {
    double d[3];
    sub3(P[k], g, d);
    r = fmax(r, sqrt(dot3d(d, d)));
  }
  sg[0][j] = make_float4((float)(a[0] - pc[0]), (float)(a[1] - pc[1]), (float)(a[2] - pc[2]),
                         l0 > 0.0 ? (float)(1.0 / l0) : 0.0f);
  sg[1][j] = make_float4((float)e0[0], (float)e0[1], (float)e0[2], l1 > 0.0 ? (float)(1.0 / l1) : 0.0f);
  sg[2][j] = make_float4((float)e1[0], (float)e1[1], (float)e1[2], l2 > 0.0 ? (float)(1.0 / l2) : 0.0f);
  sg[3][j] = make_float4((float)(U[0] * inn), (float)(U[1] * inn), (float)(U[2] * inn), 0.0f);
  sg[4][j] = make_float4((float)(V[0] * inn), (float)(V[1] * inn), (float)(V[2] * inn), 0.0f);
  sg[5][j] = make_float4((float)(n[0] * rn), (float)(n[1] * rn), (float)(n[2] * rn), 0.0f);
  sg[6][j] = make_float4((float)(g[0] - pc[0]), (float)(g[1] - pc[1]), (float)(g[2] - pc[2]),
                         (float)(r * (1.0 + 1e-6) + 1e-5));
}

__device__ __forceinline__ float geo_d2f(const float4 (*sg)[C3_LIST], int j, float px, float py, float pz) {
  const float4 g0 = sg[0][j], g1 = sg[1][j], g2 = sg[2][j], g3 = sg[3][j], g4 = sg[4][j], g5 = sg[5][j];
  const float apx = px - g0.x, apy = py - g0.y, apz = pz - g0.z;
  const float u = dot3f(apx, apy, apz, g3.x, g3.y, g3.z), v = dot3f(apx, apy, apz, g4.x, g4.y, g4.z);
  const float h = dot3f(apx, apy, apz, g5.x, g5.y, g5.z);
  float d = seg_d2f(apx, apy, apz, g1.x, g1.y, g1.z, g0.w);
  d = fminf(d, seg_d2f(apx, apy, apz, g2.x, g2.y, g2.z, g1.w));
  d = fminf(d, seg_d2f(apx - g1.x, apy - g1.y, apz - g1.z, g2.x - g1.x, g2.y - g1.y, g2.z - g1.z, g2.w));
  return (u > 0.0f && v > 0.0f && u + v < 1.0f) ? h * h : d;
}

// side of point P (true: inside) at its closest triangle tg with weights w:
// face normal, sum of the two face normals at an edge, or the angle-weighted
// vertex normal (outward for orientation o = +1)
__device__ __forceinline__ bool mesh_side(const MemDev& md, const MeshDev& mh, int tg, const double* w,
                                          const double* P, double o) {
  const int* tv = mh.tri + 3 * tg;
  double Qp[3] = {0, 0, 0}, nrm[3];
  for (int k = 0; k < 3; k++)
    for (int a = 0; a < 3; a++) Qp[a] += w[k] * md.X[3 * tv[k] + a];
  const int zeros = (w[0] == 0.0) + (w[1] == 0.0) + (w[2] == 0.0);
  if (zeros == 0) {
    for (int a = 0; a < 3; a++) nrm[a] = mh.fn[3 * tg + a];
  } else if (zeros == 1) {
    const int k = w[0] == 0.0 ? 0 : (w[1] == 0.0 ? 1 : 2);  // edge opposite vertex k
    const int nb = mh.tadj[3 * tg + (k + 1) % 3];
    for (int a = 0; a < 3; a++) nrm[a] = mh.fn[3 * tg + a] + mh.fn[3 * nb + a];
  } else {
    const int k = w[0] != 0.0 ? 0 : (w[1] != 0.0 ? 1 : 2);
    for (int a = 0; a < 3; a++) nrm[a] = mh.vn[3 * tv[k] + a];
  }
  double dv[3];
  sub3(P, Qp, dv);
  return o * dot3d(dv, nrm) < 0.0;
}

__device__ __forceinline__ double tri_d2_id(const MemDev& md, const MeshDev& mh, int tg, const double* P,
                                            double* w) {
  const int* tv = mh.tri + 3 * tg;
  return tri_d2(P, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], w);
}

// (d2, index) argmin with the lowest index on ties
__device__ __forceinline__ void argmin_merge(double& d, int& i, double d2, int i2) {
  if (d2 < d || (d2 == d && i2 >= 0 && (i < 0 || i2 < i))) {
    d = d2;
    i = i2;
  }
}

__device__ __forceinline__ void wave_argmin(double& d, int& i) {
  for (int o = 32; o > 0; o >>= 1) {
    const double d2 = __shfl_xor(d, o, 64);
    const int i2 = __shfl_xor(i, o, 64);
    argmin_merge(d, i, d2, i2);
  }
}


template <int NT>
__device__ void block_argmin(double& d, int& i, double* sd, int* si) {
  wave_argmin(d, i);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sd[wv] = d;
    si[wv] = i;
  }
  __syncthreads();
  d = sd[0];
  i = si[0];
  for (int k = 1; k < NT / 64; k++) argmin_merge(d, i, sd[k], si[k]);
  __syncthreads();
}


// one 8^3 tile at a time per workgroup of 512 threads; resident workgroups
// take the active tiles from a counter (tiles differ in cost by 20x, so a
// fixed assignment leaves CUs idle at the end); wave w holds the 4^3
// sub-tile (w & 1, (w >> 1) & 1, w >> 2)
template <class St, typename R, int NT>
__global__ __launch_bounds__(NT) void k_coupling3d(MemDev md, MeshDev mh, TileMap tm, Coup3Args ca,
                                                   const float4* __restrict__ ttab,
                                                   const float4* __restrict__ ctab,
                                                   double* __restrict__ Ifield, St cur) {
  static_assert(NT == 512, "one thread per node of an 8^3 tile");
  __shared__ float4 s_g[C3_GEO][C3_LIST];
  __shared__ int s_id[C3_IDS];
  __shared__ unsigned short s_wl[NT / 64][C3_LIST];
  __shared__ int s_cnt;
  __shared__ double s_red[NT / 64];
  __shared__ int s_redi[NT / 64];
  __shared__ float s_redf[NT / 64];
  __shared__ int b_tri[COUP3_KEEP][NT];
  __shared__ double b_sd[COUP3_KEEP][NT];
  __shared__ int s_hv[COUP3_HASH];                 // marker id of each hash slot, -1 free
  __shared__ long long s_ha[COUP3_HASH][3];        // its fixed-point force sums
  __shared__ int s_li;
  const int ntl = tm.tstate[0];
  const double reach = ca.r_cut + 1.0;
  const double hd = 0.5 * TILE3 * 1.7320508075688772;  // tile half-diagonal (box tests)
  // largest distance of a node from the centre of its tile / sub-tile
  const double rn8 = 0.5 * (TILE3 - 1) * 1.7320508075688772;
  const double rn4 = 0.5 * (TILE3 / 2 - 1) * 1.7320508075688772;
  const float mg = 0.01f;                                // FP32 distance margin
  const int per[3] = {1, !ca.wall_y, !ca.wall_z};
  const int dims[3] = {ca.nx, ca.ny, ca.nz};
  const int lt = (int)threadIdx.x, lane = lt & 63, wv = lt >> 6;
  const int off[3] = {(wv & 1) * 4 + (lane & 3), ((wv >> 1) & 1) * 4 + ((lane >> 2) & 3),
                      (wv >> 2) * 4 + (lane >> 4)};
  // sub-tile centre relative to the tile centre
  const float cwf[3] = {(wv & 1) ? 2.0f : -2.0f, ((wv >> 1) & 1) ? 2.0f : -2.0f, (wv >> 2) ? 2.0f : -2.0f};
  const unsigned long long below = (1ull << lane) - 1ull;
  for (;;) {
    // the previous tile ended with a barrier, so s_li is free to rewrite
    if (lt == 0) s_li = atomicAdd(&tm.tstate[2], 1);
    __syncthreads();
    const int li = s_li;
    if (li >= ntl) break;  // uniform over the workgroup
    const int t = tm.tlist[li];
    const int tx = t % tm.ntx, ty = (t / tm.ntx) % tm.nty, tz = t / (tm.ntx * tm.nty);
    const int t0[3] = {tx * TILE3, ty * TILE3, tz * TILE3};
    const int xi[3] = {t0[0] + off[0], t0[1] + off[1], t0[2] + off[2]};
    const bool valid = xi[0] < ca.nx && xi[1] < ca.ny && xi[2] < ca.nz;
    const long long nodeid = valid ? ((long long)xi[2] * ca.ny + xi[1]) * ca.nx + xi[0] : 0;
    // the node's cache entries of both slots, loaded before the membrane loop
    // so that their latency overlaps the tile geometry (read only for a valid
    // node inside a grown box, and only with the cache on)
    int kpre[COUP3_CACHE];
    float lpre[COUP3_CACHE];
    {
      const bool on = ca.ckey != nullptr;
      const int* kp = on ? ca.ckey : md.status;
      const float* lp = on ? ca.clb : (const float*)md.status;
#pragma unroll
      for (int c = 0; c < COUP3_CACHE; c++) {
        const long long e = on ? (long long)c * ca.N + nodeid : 0;
        kpre[c] = kp[e];
        lpre[c] = lp[e];
      }
    }
    const double ct[3] = {t0[0] + 0.5 * (TILE3 - 1), t0[1] + 0.5 * (TILE3 - 1), t0[2] + 0.5 * (TILE3 - 1)};
    double Itot = 0.0;
    int kept = 0;
    for (int m = 0; m < md.K; m++) {
      const TileGeo g = tile_geo(md.mbox + 8 * m, ct, xi, t0, dims, per, hd, reach, valid);
      if (g.miss) continue;  // uniform over the block
      const int t0m = mh.toff[m], nt = mh.toff[m + 1] - t0m;
      const double o = md.mbox[8 * m + 6];
      const int slot = kept++;
      double d2b = 1e300;
      int tb = -1;
      bool decided = false;  // I of this node already added (no band data)
      // cache: a node's entry holds while the nearest triangle of the one-ring
      // of its kept triangle (FP64, lowest index on ties) is nearer than the
      // bound less the drift since, or, beyond the band, while the bound less
      // the drift exceeds r_cut.  A tile skips the search when every node holds.
      const bool cslot = ca.ckey != nullptr && slot < COUP3_CACHE && !g.split && m < 2048;  // uniform
      const long long cix = (long long)slot * ca.N + nodeid;
      const double drift = md.mbox[8 * m + 7];
      bool cached = false;
      if (cslot) {
        bool ok = true;
        int side = -1;
        if (valid && g.inbox) {
          int key = kpre[0];
          float klb = lpre[0];
#pragma unroll
          for (int c = 1; c < COUP3_CACHE; c++)
            if (slot == c) {
              key = kpre[c];
              klb = lpre[c];
            }
          ok = key >= 0 && (key >> C3_KEYB) == m;
          if (ok) {
            const double thr = (double)klb - drift;
            const int q = key & ((1 << C3_KEYB) - 1);
            if (q >= C3_OUT) {
              ok = thr > ca.r_cut;
              side = q == C3_IN ? 1 : 0;
            } else {
              const int* tv = mh.tri + 3 * (t0m + q);
              for (int k = 0; k < 3; k++) {
                const int v = tv[k];
                for (int e = mh.vtoff[v]; e < mh.vtoff[v + 1]; e++) {
                  const int tq = mh.vt[e];
                  double w[3];
                  argmin_merge(d2b, tb, tri_d2_id(md, mh, tq, g.pp, w), tq - t0m);
                }
              }
              ok = sqrt(d2b) < thr;
            }
          }
        }
        cached = __syncthreads_and(ok) != 0;
        if (!cached) {
          d2b = 1e300;
          tb = -1;
        } else if (side >= 0) {
          Itot += side ? 1.0 : 0.0;
          decided = true;
        }
      }
      // entry written after a search (-1: none)
      int keyw = -1;
      double lbw = 0.0;
      if (cached) {
        // nothing to search
      } else if (g.split) {
        // nodes of different images: each searches the whole mesh in FP64
        if (g.inbox)
          for (int q = 0; q < nt; q++) {
            double w[3];
            argmin_merge(d2b, tb, tri_d2_id(md, mh, t0m + q, g.pp, w), q);
          }
      } else {
        const double* bx = md.mbox + 8 * m;
        const float pcr[3] = {(float)(g.pc[0] - 0.5 * (bx[0] + bx[3])), (float)(g.pc[1] - 0.5 * (bx[1] + bx[4])),
                              (float)(g.pc[2] - 0.5 * (bx[2] + bx[5]))};
        const float4* tab = ttab + 4 * (size_t)t0m;
        const float4* cls = ctab + mh.coff[m];
        const int ncl = mh.coff[m + 1] - mh.coff[m];
        // distance of the tile centre to the mesh: the least cluster upper
        // bound, then exact distances in the clusters that reach below it
        // (one wave per cluster, one lane per triangle)
        float ul = 3.0e38f;
        for (int k = lt; k < ncl; k += NT) ul = fminf(ul, sph_dist(pcr[0], pcr[1], pcr[2], cls[k]) + cls[k].w);
        const float U = block_minf<NT>(ul, s_redf) + mg;
        float dl = 3.0e38f;
        for (int k = wv; k < ncl; k += NT / 64) {
          const float4 cs = cls[k];
          if (sph_dist(pcr[0], pcr[1], pcr[2], cs) - cs.w > U) continue;
          const int q = k * CL3 + lane;
          if (q < nt) dl = fminf(dl, tri_d2f_vtx(pcr[0], pcr[1], pcr[2], tab[4 * q], tab[4 * q + 1], tab[4 * q + 2]));
        }
        const float dminf = sqrtf(block_minf<NT>(dl, s_redf));
        if ((double)dminf > ca.r_cut + rn8 + 0.02 + (cslot ? COUP3_BEYOND : 0.0f)) {
          // the whole tile is beyond r_cut: every node is on the side of the
          // tile centre, taken at the centre's closest triangle
          const float tl = dminf * dminf + 0.05f + 1e-4f * dminf * dminf;
          const float tlr = sqrtf(tl) + mg;
          double dc = 1e300;
          int ic = -1;
          for (int k = wv; k < ncl; k += NT / 64) {
            const float4 cs = cls[k];
            if (sph_dist(pcr[0], pcr[1], pcr[2], cs) - cs.w > tlr) continue;
            const int q = k * CL3 + lane;
            if (q < nt &&
                tri_d2f_vtx(pcr[0], pcr[1], pcr[2], tab[4 * q], tab[4 * q + 1], tab[4 * q + 2]) <= tl) {
              double w[3];
              argmin_merge(dc, ic, tri_d2_id(md, mh, t0m + q, g.pc, w), q);
            }
          }
          block_argmin<NT>(dc, ic, s_red, s_redi);
          if (ic >= 0) {  // always: the FP32 minimum itself is within tl
            double w[3];
            tri_d2_id(md, mh, t0m + ic, g.pc, w);
            const bool in = mesh_side(md, mh, t0m + ic, w, g.pc, o);
            if (g.inbox && in) Itot += 1.0;
            if (cslot && valid && g.inbox) {
              // every node is at least dmin - rn8 from the mesh, on the centre's side
              keyw = (m << C3_KEYB) | (in ? C3_IN : C3_OUT);
              lbw = (double)dminf - rn8 - 0.02 - 1e-4 * (double)dminf;
            }
          }
          decided = true;
        } else {
          // tile candidates: every node's closest triangle lies within
          // dmin + 2 rn8 of the tile centre.  Their ids go to LDS; their
          // geometry is staged C3_LIST at a time.
          const float cull = dminf + (float)(2.0 * rn8) + 0.02f + (cslot ? COUP3_PAD : 0.0f);
          if (lt == 0) s_cnt = 0;
          __syncthreads();
          for (int k = wv; k < ncl; k += NT / 64) {
            const float4 cs = cls[k];
            if (sph_dist(pcr[0], pcr[1], pcr[2], cs) - cs.w > cull) continue;
            const int q = k * CL3 + lane;
            bool in = false;
            if (q < nt) {
              const float4 sp = tab[4 * q + 3];
              const float dc = sph_dist(pcr[0], pcr[1], pcr[2], sp);
              in = dc - sp.w <= cull &&
                   (dc + sp.w <= cull ||
                    tri_d2f_vtx(pcr[0], pcr[1], pcr[2], tab[4 * q], tab[4 * q + 1], tab[4 * q + 2]) <= cull * cull);
            }
            const unsigned long long mk = __ballot(in);
            int base = 0;
            if (lane == 0 && mk) base = atomicAdd(&s_cnt, __popcll(mk));
            base = __shfl(base, 0, 64);
            const int j = base + __popcll(mk & below);
            if (in && j < C3_IDS) s_id[j] = q;
          }
          __syncthreads();
          const int nc = s_cnt;
          if (nc > C3_IDS) {
            // more candidates than ids fit: chunks of the whole mesh, every
            // node re-evaluating the chunk's candidates in FP64
            for (int c0 = 0; c0 < nt; c0 += C3_IDS) {
              __syncthreads();
              if (lt == 0) s_cnt = 0;
              __syncthreads();
              for (int q = c0 + lt; q < min(nt, c0 + C3_IDS); q += NT)
                if (tri_d2f_vtx(pcr[0], pcr[1], pcr[2], tab[4 * q], tab[4 * q + 1], tab[4 * q + 2]) <= cull * cull)
                  s_id[atomicAdd(&s_cnt, 1)] = q;
              __syncthreads();
              const int ncc = s_cnt;
              if (g.inbox)
                for (int j = 0; j < ncc; j++) {
                  double w[3];
                  argmin_merge(d2b, tb, tri_d2_id(md, mh, t0m + s_id[j], g.pp, w), s_id[j]);
                }
            }
          } else {
            const int nch = (nc + C3_LIST - 1) / C3_LIST;
            // stage the geometry of chunk c (all threads; the caller syncs)
            auto stage = [&](int c) {
              const int c0 = c * C3_LIST, n0 = min(C3_LIST, nc - c0);
              for (int j = lt; j < n0; j += NT) {
                const int* tv = mh.tri + 3 * (t0m + s_id[c0 + j]);
                geo_store(s_g, j, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], g.pc);
              }
            };
            // 1. sub-tile centre distance over all candidates (the least
            //    upper bound so far gates the exact distances)
            float dw = 3.0e38f, uw = 3.0e38f;
            for (int c = 0; c < nch; c++) {
              __syncthreads();
              stage(c);
              __syncthreads();
              const int n0 = min(C3_LIST, nc - c * C3_LIST);
              float u = uw;
              for (int j = lane; j < n0; j += 64) u = fminf(u, sph_dist(cwf[0], cwf[1], cwf[2], s_g[6][j]) + s_g[6][j].w);
              uw = wave_minf(u);
              // entries whose sphere reaches below uw, compacted, then exact
              int ne = 0;
              for (int base = 0; base < n0; base += 64) {
                const int j = base + lane;
                const bool pr = j < n0 && sph_dist(cwf[0], cwf[1], cwf[2], s_g[6][j]) - s_g[6][j].w <= uw + mg;
                const unsigned long long mk = __ballot(pr);
                if (pr) s_wl[wv][ne + __popcll(mk & below)] = (unsigned short)j;
                ne += __popcll(mk);
              }
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              __builtin_amdgcn_wave_barrier();
              for (int k = lane; k < ne; k += 64) dw = fminf(dw, geo_d2f(s_g, s_wl[wv][k], cwf[0], cwf[1], cwf[2]));
              __builtin_amdgcn_wave_barrier();
            }
            dw = wave_minf(dw);
            const float dwr = sqrtf(dw);
            // the whole sub-tile beyond r_cut: the side of its centre
            const bool wfar = (double)dwr > ca.r_cut + rn4 + 0.01 + (cslot ? COUP3_BEYOND : 0.0f);  // uniform over the wave
            const double pw[3] = {g.pc[0] + cwf[0], g.pc[1] + cwf[1], g.pc[2] + cwf[2]};
            const float tlw = dw + 0.05f + 1e-4f * dw;
            const float tlwr = sqrtf(tlw) + mg;
            const float cwr = dwr + (float)(2.0 * rn4) + mg + (cslot ? COUP3_PAD : 0.0f);
            const float pn[3] = {(float)(g.pp[0] - g.pc[0]), (float)(g.pp[1] - g.pc[1]), (float)(g.pp[2] - g.pc[2])};
            // the sub-tile's share of chunk c (bounding spheres within reach),
            // compacted with ballots
            auto wave_list = [&](int c) {
              const int n0 = min(C3_LIST, nc - c * C3_LIST);
              int cnt = 0;
              for (int base = 0; base < n0; base += 64) {
                const int j = base + lane;
                const bool pr = j < n0 && sph_dist(cwf[0], cwf[1], cwf[2], s_g[6][j]) - s_g[6][j].w <= cwr;
                const unsigned long long mk = __ballot(pr);
                if (pr) s_wl[wv][cnt + __popcll(mk & below)] = (unsigned short)j;
                cnt += __popcll(mk);
              }
              __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
              __builtin_amdgcn_wave_barrier();
              return cnt;
            };
            // 2. far sub-tiles: FP64 near-ties of the centre; near ones: the
            //    FP32 minimum of every node
            double dc = 1e300;
            int ic = -1;
            float bf = 3.0e38f;
            int cnt = 0;
            // entries that were within the tie tolerance of the node's
            // running FP32 minimum when scanned (a superset of its final
            // near-ties), one bit per wave-list entry
            unsigned long long msk[C3_LIST / 64];
#pragma unroll
            for (int w = 0; w < C3_LIST / 64; w++) msk[w] = 0ull;
            for (int c = 0; c < nch; c++) {
              if (nch > 1) {
                __syncthreads();
                stage(c);
                __syncthreads();
              }
              const int c0 = c * C3_LIST, n0 = min(C3_LIST, nc - c0);
              if (wfar) {
                for (int j = lane; j < n0; j += 64) {
                  if (sph_dist(cwf[0], cwf[1], cwf[2], s_g[6][j]) - s_g[6][j].w > tlwr) continue;
                  if (geo_d2f(s_g, j, cwf[0], cwf[1], cwf[2]) <= tlw) {
                    double w[3];
                    argmin_merge(dc, ic, tri_d2_id(md, mh, t0m + s_id[c0 + j], pw, w), s_id[c0 + j]);
                  }
                }
              } else {
                cnt = wave_list(c);
                if (g.inbox && nch == 1) {
#pragma unroll
                  for (int w = 0; w < C3_LIST / 64; w++) {
                    const int k0 = w * 64, k1 = min(cnt, k0 + 64);
                    unsigned long long mw = 0ull;
                    for (int k = k0; k < k1; k++) {
                      const float d = geo_d2f(s_g, s_wl[wv][k], pn[0], pn[1], pn[2]);
                      bf = fminf(bf, d);
                      mw |= (d <= bf + 1e-3f + 1e-5f * bf ? 1ull : 0ull) << (k - k0);
                    }
                    msk[w] = mw;
                  }
                } else if (g.inbox) {
                  for (int k = 0; k < cnt; k++) bf = fminf(bf, geo_d2f(s_g, s_wl[wv][k], pn[0], pn[1], pn[2]));
                }
              }
            }
            if (wfar) {
              wave_argmin(dc, ic);
              if (ic >= 0) {  // always: the FP32 minimum itself is within tlw
                double w[3];
                tri_d2_id(md, mh, t0m + ic, pw, w);
                const bool in = mesh_side(md, mh, t0m + ic, w, pw, o);
                if (g.inbox && in) Itot += 1.0;
                if (cslot && valid && g.inbox) {
                  keyw = (m << C3_KEYB) | (in ? C3_IN : C3_OUT);
                  lbw = (double)dwr - rn4 - 0.01 - 1e-4 * (double)dwr;
                }
              }
              decided = true;
            }
            // 3. near sub-tiles: FP64 re-evaluation of every candidate within
            //    the FP32 rounding margin of the node's minimum
            const float tol = 1e-3f + 1e-5f * bf;
            const float tolr = sqrtf(bf + tol) + mg;
            for (int c = 0; c < nch; c++) {
              if (nch > 1) {
                __syncthreads();
                stage(c);
                __syncthreads();
              }
              if (!wfar) {
                const int c0 = c * C3_LIST;
                if (nch > 1) cnt = wave_list(c);
                // each node first collects its own near-ties (in registers),
                // then all lanes re-evaluate theirs together, so the wave runs
                // as many FP64 evaluations as the largest tie set, not as the
                // union of all its nodes' ties
                int tie[C3_TIES];
                int nti = 0;
                bool more = false;
                auto add_tie = [&](int q) {
#pragma unroll
                  for (int r = 0; r < C3_TIES; r++)
                    if (r == nti) tie[r] = q;
                  more |= nti == C3_TIES;
                  nti += nti < C3_TIES;
                };
                if (g.inbox && nch == 1) {
                  // only the entries marked in the first scan
#pragma unroll
                  for (int w = 0; w < C3_LIST / 64; w++) {
                    unsigned long long mw = msk[w];
                    while (mw) {
                      const int k = w * 64 + __ffsll((long long)mw) - 1;
                      mw &= mw - 1ull;
                      const int j = s_wl[wv][k];
                      if (geo_d2f(s_g, j, pn[0], pn[1], pn[2]) <= bf + tol) add_tie(s_id[j]);
                    }
                  }
                } else if (g.inbox) {
                  for (int k = 0; k < cnt; k++) {
                    const int j = s_wl[wv][k];
                    const float4 sp = s_g[6][j];
                    if (sph_dist(pn[0], pn[1], pn[2], sp) - sp.w > tolr) continue;
                    if (geo_d2f(s_g, j, pn[0], pn[1], pn[2]) > bf + tol) continue;
                    add_tie(s_id[c0 + j]);
                  }
                }
#pragma unroll
                for (int r = 0; r < C3_TIES; r++)
                  if (r < nti) {
                    double w[3];
                    argmin_merge(d2b, tb, tri_d2_id(md, mh, t0m + tie[r], g.pp, w), tie[r]);
                  }
                if (more)  // more ties than registers: every candidate again
                  for (int k = 0; k < cnt; k++) {
                    const int j = s_wl[wv][k];
                    if (geo_d2f(s_g, j, pn[0], pn[1], pn[2]) > bf + tol) continue;
                    double w[3];
                    argmin_merge(d2b, tb, tri_d2_id(md, mh, t0m + s_id[c0 + j], g.pp, w), s_id[c0 + j]);
                  }
              }
            }
            // several chunks: once every node's closest triangle is known,
            // the chunks are staged again to bound the listed triangles that
            // share no vertex with it (one chunk: still staged, below)
            float o2m = 3.0e38f;
            if (cslot && nch > 1) {  // uniform over the block
              int v0 = -1, v1 = -1, v2 = -1;
              if (valid && g.inbox && tb >= 0) {
                const int* tv = mh.tri + 3 * (t0m + tb);
                v0 = tv[0];
                v1 = tv[1];
                v2 = tv[2];
              }
              for (int c = 0; c < nch; c++) {
                __syncthreads();
                stage(c);
                __syncthreads();
                if (!wfar) {
                  const int c0 = c * C3_LIST, cn = wave_list(c);
                  if (v0 >= 0)
                    for (int k = 0; k < cn; k++) {
                      const int j = s_wl[wv][k];
                      const int* uv = mh.tri + 3 * (t0m + s_id[c0 + j]);
                      bool adj = false;
#pragma unroll
                      for (int a = 0; a < 3; a++) adj |= uv[a] == v0 || uv[a] == v1 || uv[a] == v2;
                      if (!adj) o2m = fminf(o2m, geo_d2f(s_g, j, pn[0], pn[1], pn[2]));
                    }
                }
              }
            }
            if (cslot && !wfar && valid && g.inbox && tb >= 0) {
              const double d = sqrt(d2b);
              if (d > ca.r_cut + COUP3_BEYOND) {
                // well beyond the band: keep the side and the distance
                double w[3];
                tri_d2_id(md, mh, t0m + tb, g.pp, w);
                keyw = (m << C3_KEYB) | (mesh_side(md, mh, t0m + tb, w, g.pp, o) ? C3_IN : C3_OUT);
                lbw = d;
              } else {
                // triangles off the sub-tile's list lie farther than cwr from
                // its centre and those off the tile's list farther than cull
                // from the tile centre; listed ones that share no vertex with
                // tb are bounded by their FP32 distance less its rounding
                float o2 = o2m;
                if (nch == 1) {
                  const int* tv = mh.tri + 3 * (t0m + tb);
                  const int v0 = tv[0], v1 = tv[1], v2 = tv[2];
                  for (int k = 0; k < cnt; k++) {
                    const int j = s_wl[wv][k];
                    const int* uv = mh.tri + 3 * (t0m + s_id[j]);
                    bool adj = false;
#pragma unroll
                    for (int a = 0; a < 3; a++) adj |= uv[a] == v0 || uv[a] == v1 || uv[a] == v2;
                    if (!adj) o2 = fminf(o2, geo_d2f(s_g, j, pn[0], pn[1], pn[2]));
                  }
                }
                const double lout = fmin((double)cwr - rn4 - 0.01, (double)cull - rn8 - 0.02);
                keyw = (m << C3_KEYB) | tb;
                lbw = fmin(sqrt(fmax((double)o2 - (1e-3 + 1e-5 * (double)o2), 0.0)), lout);
              }
            }
          }
        }
      }
      if (cslot && !cached && valid) {
        // FP32 distances are within 1e-5 relative of exact here: a margin of
        // 1e-3 plus 1e-5 of the bound; stored with the drift so far added and
        // rounded down, so the bound at a later step is the stored value less
        // the drift then
        ca.ckey[cix] = keyw;
        ca.clb[cix] = keyw >= 0 ? __double2float_rd(lbw - 1e-3 - 1e-5 * fabs(lbw) + drift) : 0.0f;
      }
      double sd = 0.0;
      bool band = false;
      if (!decided && g.inbox && tb >= 0) {
        double w[3];
        tri_d2_id(md, mh, t0m + tb, g.pp, w);
        const bool in = mesh_side(md, mh, t0m + tb, w, g.pp, o);
        const double d = sqrt(d2b);
        sd = in ? d : -d;
        band = d <= ca.r_cut;
        Itot += band ? 0.5 * (1.0 + tanh(sd / (2.0 * ca.alpha))) : (in ? 1.0 : 0.0);
      }
      if (slot < COUP3_KEEP) {
        b_tri[slot][lt] = band ? t0m + tb : -1;
        b_sd[slot][lt] = sd;
      }
      __syncthreads();  // candidate lists are rebuilt for the next membrane
    }
    const long long node = valid ? ((long long)xi[2] * ca.ny + xi[1]) * ca.nx + xi[0] : 0;
    if (valid) Ifield[node] = Itot;
    if (ca.want_force) {
      if (kept > COUP3_KEEP && lt == 0) md.status[1] = 1;
      bool anyband = false;
      for (int k = 0; k < min(kept, COUP3_KEEP); k++) anyband |= b_tri[k][lt] >= 0;
      // psi and the force pass only in waves that hold band nodes
      double psi = 0.0;
      const bool wband = __ballot(anyband) != 0ull;
      if (valid && wband) {
        using L = Lattice<19>;
        psi = cur.rest(2, node);
        // neighbour planes, rows and columns of the node, wrapped once
        const long long pl = (long long)ca.ny * ca.nx;
        const long long zlo = (xi[2] == 0 ? ca.nz - 1 : xi[2] - 1) * pl, zc = xi[2] * pl;
        const long long zhi = (xi[2] == ca.nz - 1 ? 0 : xi[2] + 1) * pl;
        const long long ylo = (long long)(xi[1] == 0 ? ca.ny - 1 : xi[1] - 1) * ca.nx;
        const long long yhi = (long long)(xi[1] == ca.ny - 1 ? 0 : xi[1] + 1) * ca.nx;
        const long long yc = (long long)xi[1] * ca.nx;
        const int xlo = xi[0] == 0 ? ca.nx - 1 : xi[0] - 1, xhi = xi[0] == ca.nx - 1 ? 0 : xi[0] + 1;
        const bool wylo = ca.wall_y && xi[1] == 0, wyhi = ca.wall_y && xi[1] == ca.ny - 1;
        const bool wzlo = ca.wall_z && xi[2] == 0, wzhi = ca.wall_z && xi[2] == ca.nz - 1;
        for (int i = 1; i < 19; i++) {
          const int ex = L::cx[i], ey = L::cy[i], ez = L::cz[i];
          const bool back = (ey > 0 ? wylo : (ey < 0 ? wyhi : false)) || (ez > 0 ? wzlo : (ez < 0 ? wzhi : false));
          const long long sn = (ez > 0 ? zlo : (ez < 0 ? zhi : zc)) + (ey > 0 ? ylo : (ey < 0 ? yhi : yc)) +
                               (ex > 0 ? xlo : (ex < 0 ? xhi : xi[0]));
          psi += (double)cur.template load<R>(2, back ? L::opp[i] : i, back ? node : sn);
        }
      }
      // an empty hash table (the previous tile flushed it before its last barrier)
      for (int i = lt; i < COUP3_HASH; i += NT) {
        s_hv[i] = -1;
        s_ha[i][0] = s_ha[i][1] = s_ha[i][2] = 0;
      }
      __syncthreads();
      int slot = 0;
      for (int m = 0; wband && m < md.K && slot < COUP3_KEEP; m++) {
        const TileGeo g = tile_geo(md.mbox + 8 * m, ct, xi, t0, dims, per, hd, reach, valid);
        if (g.miss) continue;
        const int my = slot++;
        const int tg = b_tri[my][lt];
        if (tg < 0) continue;
        const double sd = b_sd[my][lt];
        const double d = fabs(sd);
        if (d == 0.0) continue;
        double w[3];
        tri_d2_id(md, mh, tg, g.pp, w);
        const int* tv = mh.tri + 3 * tg;
        double Qp[3] = {0, 0, 0};
        for (int k = 0; k < 3; k++)
          for (int a = 0; a < 3; a++) Qp[a] += w[k] * md.X[3 * tv[k] + a];
        const double sg = sd > 0.0 ? 1.0 : -1.0;
        const double ch = cosh(sd / (2.0 * ca.alpha));
        const double wgt = ca.kappa_c / (4.0 * ca.alpha) * (psi - Itot) / (ch * ch);
        for (int k = 0; k < 3; k++) {
          const int v = tv[k];
          long long fx[3];
          for (int a = 0; a < 3; a++) fx[a] = to_fix(-sg * (g.pp[a] - Qp[a]) / d * wgt * w[k]);
          // slot of marker v: linear probing from its hash
          int h = (int)(((unsigned)v * 2654435761u) >> 23) & (COUP3_HASH - 1);
          int found = -1;
          for (int probe = 0; probe < COUP3_HASH; probe++) {
            const int prev = atomicCAS(&s_hv[h], -1, v);
            if (prev == -1 || prev == v) {
              found = h;
              break;
            }
            h = (h + 1) & (COUP3_HASH - 1);
          }
          if (found >= 0) {
            for (int a = 0; a < 3; a++) atomicAdd((unsigned long long*)&s_ha[found][a], (unsigned long long)fx[a]);
          } else {
            long long* A = md.Facc + 3 * v;
            for (int a = 0; a < 3; a++) atomicAdd((unsigned long long*)&A[a], (unsigned long long)fx[a]);
          }
        }
      }
      __syncthreads();
      // one global atomic per marker and component (integer sums: the same
      // totals in any order)
      for (int i = lt; i < COUP3_HASH; i += NT) {
        const int v = s_hv[i];
        if (v >= 0) {
          long long* A = md.Facc + 3 * v;
          for (int a = 0; a < 3; a++)
            if (s_ha[i][a] != 0) atomicAdd((unsigned long long*)&A[a], (unsigned long long)s_ha[i][a]);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// edge springs and dihedral bending, one thread per edge, forces added to
// the fixed-point accumulators of the markers (order independent)
__device__ __forceinline__ void acc_force(long long* Facc, int v, const double* f) {
  for (int a = 0; a < 3; a++)
    atomicAdd((unsigned long long*)&Facc[3 * v + a], (unsigned long long)to_fix(f[a]));
}

// gradient of s with respect to the three vertices of a triangle whose
// (unnormalised) area vector is n = (p1 - p0) x (p2 - p0), given ds/dn
__device__ __forceinline__ void area_grad(const double* p0, const double* p1, const double* p2,
                                          const double* dsdn, double* g0, double* g1, double* g2) {
  double e1[3], e2[3];
  sub3(p1, p0, e1);
  sub3(p2, p0, e2);
  cross3d(e2, dsdn, g1);   // ds/dp1 = e2 x ds/dn
  cross3d(dsdn, e1, g2);   // ds/dp2 = ds/dn x e1
  for (int a = 0; a < 3; a++) g0[a] = -g1[a] - g2[a];
}

__global__ void k_memedge3d(MemDev md, MeshDev mh, const int* __restrict__ emem) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mh.E) return;
  const int m = emem[e];
  const double ks = md.ks[m], kb = md.kb[m];
  const int a = mh.edge[4 * e], b = mh.edge[4 * e + 1], t1 = mh.edge[4 * e + 2], t2 = mh.edge[4 * e + 3];
  const double* pa = md.X + 3 * a;
  const double* pb = md.X + 3 * b;
  // spring: E = ks/2 (l/l0 - 1)^2 l0 (meshes with a triangle law instead
  // take their strain energy from k_memtri3d)
  if (md.law[m] == 0) {
    double dvec[3];
    sub3(pb, pa, dvec);
    const double len = sqrt(dot3d(dvec, dvec));
    const double s = ks * (len / mh.erest[e] - 1.0) / len;
    double fb[3] = {-s * dvec[0], -s * dvec[1], -s * dvec[2]};
    double fa[3] = {-fb[0], -fb[1], -fb[2]};
    acc_force(md.Facc, a, fa);
    acc_force(md.Facc, b, fb);
  }
  if (kb == 0.0) return;
  // dihedral: E = kb (1 - n1.n2 / (|n1| |n2|))
  const int* v1 = mh.tri + 3 * t1;
  const int* v2 = mh.tri + 3 * t2;
  double n1[3], n2[3], e1[3], e2[3];
  sub3(md.X + 3 * v1[1], md.X + 3 * v1[0], e1);
  sub3(md.X + 3 * v1[2], md.X + 3 * v1[0], e2);
  cross3d(e1, e2, n1);
  sub3(md.X + 3 * v2[1], md.X + 3 * v2[0], e1);
  sub3(md.X + 3 * v2[2], md.X + 3 * v2[0], e2);
  cross3d(e1, e2, n2);
  const double l1 = sqrt(dot3d(n1, n1)), l2 = sqrt(dot3d(n2, n2));
  const double c = dot3d(n1, n2) / (l1 * l2);
  double d1[3], d2[3];  // dE/dn1, dE/dn2
  for (int q = 0; q < 3; q++) {
    d1[q] = -kb * (n2[q] / (l1 * l2) - c * n1[q] / (l1 * l1));
    d2[q] = -kb * (n1[q] / (l1 * l2) - c * n2[q] / (l2 * l2));
  }
  double g0[3], g1[3], g2[3];
  area_grad(md.X + 3 * v1[0], md.X + 3 * v1[1], md.X + 3 * v1[2], d1, g0, g1, g2);
  for (int q = 0; q < 3; q++) {
    g0[q] = -g0[q];
    g1[q] = -g1[q];
    g2[q] = -g2[q];
  }
  acc_force(md.Facc, v1[0], g0);
  acc_force(md.Facc, v1[1], g1);
  acc_force(md.Facc, v1[2], g2);
  area_grad(md.X + 3 * v2[0], md.X + 3 * v2[1], md.X + 3 * v2[2], d2, g0, g1, g2);
  for (int q = 0; q < 3; q++) {
    g0[q] = -g0[q];
    g1[q] = -g1[q];
    g2[q] = -g2[q];
  }
  acc_force(md.Facc, v2[0], g0);
  acc_force(md.Facc, v2[1], g1);
  acc_force(md.Facc, v2[2], g2);
}

// Hyperelastic triangle laws: a flat triangle maps linearly from its rest
// shape (the rest lengths a_k of the edges opposite its vertices) to its
// current shape.  Invariants I1 = l1^2 + l2^2 = sum_k q_k |e_k|^2 with
// q_k = cot(rest angle k) / (2 A0), and J = l1 l2 = A / A0.  Energy A0 W
// with shear modulus G = ks: neo-Hookean W = G/2 (I1 + J^-2 - 3), Skalak
// W = G/4 ((I1-2)^2 + 2 (I1-2) - 2 (J^2-1) + C (J^2-1)^2), C = 1.
// Returns the energy; with f != nullptr also the forces -dE/dp_k.
__device__ __forceinline__ double tri_law(int law, double G, const double* p0, const double* p1,
                                          const double* p2, const double* a, double (*f)[3]) {
  const double a2[3] = {a[0] * a[0], a[1] * a[1], a[2] * a[2]};
  const double A0 = 0.25 * sqrt(2.0 * (a2[0] * a2[1] + a2[1] * a2[2] + a2[2] * a2[0]) - a2[0] * a2[0] -
                                a2[1] * a2[1] - a2[2] * a2[2]);
  const double* P[3] = {p0, p1, p2};
  double ev[3][3], q[3], I1 = 0.0;  // ev[k]: edge opposite vertex k, from vertex k+1 to k+2
  for (int k = 0; k < 3; k++) {
    sub3(P[(k + 2) % 3], P[(k + 1) % 3], ev[k]);
    q[k] = (a2[(k + 1) % 3] + a2[(k + 2) % 3] - a2[k]) / (8.0 * A0 * A0);
    I1 += q[k] * dot3d(ev[k], ev[k]);
  }
  double e1[3], e2[3], n[3];
  sub3(p1, p0, e1);
  sub3(p2, p0, e2);
  cross3d(e1, e2, n);
  const double ln = sqrt(dot3d(n, n));
  const double J = 0.5 * ln / A0;
  double W, WI, WJ;  // W and its derivatives in I1 and J
  if (law == 1) {
    W = 0.5 * G * (I1 + 1.0 / (J * J) - 3.0);
    WI = 0.5 * G;
    WJ = -G / (J * J * J);
  } else {
    const double i1 = I1 - 2.0, k2 = J * J - 1.0;
    W = 0.25 * G * (i1 * i1 + 2.0 * i1 - 2.0 * k2 + k2 * k2);
    WI = 0.5 * G * (i1 + 1.0);
    WJ = G * J * (k2 - 1.0);
  }
  if (f) {
    // d|e_k|^2: +2 e_k at vertex k+2, -2 e_k at vertex k+1
    for (int k = 0; k < 3; k++)
      for (int d = 0; d < 3; d++) f[k][d] = 0.0;
    for (int k = 0; k < 3; k++)
      for (int d = 0; d < 3; d++) {
        const double g = 2.0 * A0 * WI * q[k] * ev[k][d];
        f[(k + 2) % 3][d] -= g;
        f[(k + 1) % 3][d] += g;
      }
    // dJ = dA / A0, dA/dn = n / (2 |n|); times A0 cancels
    double dsdn[3];
    for (int d = 0; d < 3; d++) dsdn[d] = WJ * n[d] / (2.0 * ln);
    double g0[3], g1[3], g2[3];
    area_grad(p0, p1, p2, dsdn, g0, g1, g2);
    for (int d = 0; d < 3; d++) {
      f[0][d] -= g0[d];
      f[1][d] -= g1[d];
      f[2][d] -= g2[d];
    }
  }
  return A0 * W;
}

// one thread per triangle of every mesh with a triangle law
__global__ void k_memtri3d(MemDev md, MeshDev mh) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mh.T) return;
  int lo = 0, hi = md.K - 1;  // mesh of triangle t: toff[m] <= t < toff[m + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mh.toff[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int law = md.law[lo];
  if (law == 0) return;
  const int* v = mh.tri + 3 * t;
  const double a[3] = {mh.erest[mh.tedge[3 * t]], mh.erest[mh.tedge[3 * t + 1]], mh.erest[mh.tedge[3 * t + 2]]};
  double f[3][3];
  tri_law(law, md.ks[lo], md.X + 3 * v[0], md.X + 3 * v[1], md.X + 3 * v[2], a, f);
  for (int k = 0; k < 3; k++) acc_force(md.Facc, v[k], f[k]);
}

// total force per marker from the accumulators
__global__ void k_memforce3d(MemDev md) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= md.M) return;
  long long* acc = md.Facc + 3 * g;
  bool bad = false;
  for (int a = 0; a < 3; a++) {
    const double f = from_fix(acc[a]);
    acc[a] = 0;
    if (!(fabs(f) < FIX_LIMIT)) bad = true;
    md.F[3 * g + a] = f;
  }
  if (bad) md.status[0] = 1;
}

// per-edge energies (strain, bending) for the FP64 readout
__global__ void k_memenergy3d(MemDev md, MeshDev mh, const int* __restrict__ emem,
                              double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mh.E) return;
  const int m = emem[e];
  const int a = mh.edge[4 * e], b = mh.edge[4 * e + 1], t1 = mh.edge[4 * e + 2], t2 = mh.edge[4 * e + 3];
  if (md.law[m] == 0) {
    double dvec[3];
    sub3(md.X + 3 * b, md.X + 3 * a, dvec);
    const double len = sqrt(dot3d(dvec, dvec));
    const double st = len / mh.erest[e] - 1.0;
    out[2 * e] = 0.5 * md.ks[m] * st * st * mh.erest[e];
  } else {
    // a third of each adjacent triangle's energy (every triangle has three edges)
    double es = 0.0;
    for (int side = 0; side < 2; side++) {
      const int t = side ? t2 : t1;
      const int* v = mh.tri + 3 * t;
      const double ar[3] = {mh.erest[mh.tedge[3 * t]], mh.erest[mh.tedge[3 * t + 1]],
                            mh.erest[mh.tedge[3 * t + 2]]};
      es += tri_law(md.law[m], md.ks[m], md.X + 3 * v[0], md.X + 3 * v[1], md.X + 3 * v[2], ar, nullptr);
    }
    out[2 * e] = es / 3.0;
  }
  out[2 * e + 1] = md.kb[m] * (1.0 - dot3d(mh.fn + 3 * t1, mh.fn + 3 * t2));
}

// spreading, one wave per marker (lane = stencil node of the 4^3 kernel)
__global__ void k_spread3d(MemDev md, long long* __restrict__ fib, int nx, int ny, int nz, int wall_y,
                           int wall_z) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = (int)(tid >> 6), k = (int)(tid & 63);
  if (g >= md.M) return;
  const double X = md.X[3 * g], Y = md.X[3 * g + 1], Z = md.X[3 * g + 2];
  const int cx = (int)floor(X) - 1 + (k & 3), cy = (int)floor(Y) - 1 + ((k >> 2) & 3),
            cz = (int)floor(Z) - 1 + (k >> 4);
  if ((wall_y && (cy < 0 || cy >= ny)) || (wall_z && (cz < 0 || cz >= nz))) return;
  const double w = peskin(cx - X) * peskin(cy - Y) * peskin(cz - Z);
  const long long node = ((long long)wrap(cz, nz) * ny + wrap(cy, ny)) * nx + wrap(cx, nx);
  for (int a = 0; a < 3; a++)
    atomicAdd((unsigned long long*)&fib[3 * node + a], (unsigned long long)to_fix(md.F[3 * g + a] * w));
}

// interpolation of v* = u(t+1) + f(t)/(2 rho(t+1)) and Euler update, one
// wave per marker, lanes summed in a fixed butterfly order
template <class St, typename R>
__global__ void k_interp3d(MemDev md, St cur, LBParams P, const double* __restrict__ force) {
  using L = Lattice<19>;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g = (int)(tid >> 6), k = (int)(tid & 63);
  const bool live = g < md.M;
  double U[3] = {0, 0, 0}, X[3] = {0, 0, 0};
  if (live) {
    for (int a = 0; a < 3; a++) X[a] = md.X[3 * g + a];
    const int cx = (int)floor(X[0]) - 1 + (k & 3), cy = (int)floor(X[1]) - 1 + ((k >> 2) & 3),
              cz = (int)floor(X[2]) - 1 + (k >> 4);
    if (!((P.wall_y && (cy < 0 || cy >= P.ny)) || (P.wall_z && (cz < 0 || cz >= P.nz)))) {
      const int xw = wrap(cx, P.nx), yw = wrap(cy, P.ny), zw = wrap(cz, P.nz);
      const long long node = ((long long)zw * P.ny + yw) * P.nx + xw;
      // neighbour planes, rows and columns of the stencil node, wrapped once
      const long long pl = (long long)P.ny * P.nx;
      const long long zlo = (zw == 0 ? P.nz - 1 : zw - 1) * pl, zc = zw * pl;
      const long long zhi = (zw == P.nz - 1 ? 0 : zw + 1) * pl;
      const long long ylo = (long long)(yw == 0 ? P.ny - 1 : yw - 1) * P.nx;
      const long long yhi = (long long)(yw == P.ny - 1 ? 0 : yw + 1) * P.nx, yc = (long long)yw * P.nx;
      const int xlo = xw == 0 ? P.nx - 1 : xw - 1, xhi = xw == P.nx - 1 ? 0 : xw + 1;
      const bool wylo = P.wall_y && yw == 0, wyhi = P.wall_y && yw == P.ny - 1;
      const bool wzlo = P.wall_z && zw == 0, wzhi = P.wall_z && zw == P.nz - 1;
      double d = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < 19; i++) {
        const int ex = L::cx[i], ey = L::cy[i], ez = L::cz[i];
        const bool back = (ey > 0 ? wylo : (ey < 0 ? wyhi : false)) || (ez > 0 ? wzlo : (ez < 0 ? wzhi : false));
        const long long sn = (ez > 0 ? zlo : (ez < 0 ? zhi : zc)) + (ey > 0 ? ylo : (ey < 0 ? yhi : yc)) +
                             (ex > 0 ? xlo : (ex < 0 ? xhi : xw));
        const double v = (double)cur.template load<R>(0, back ? L::opp[i] : i, back ? node : sn);
        d += v;
        j[0] += L::cx[i] * v;
        j[1] += L::cy[i] * v;
        j[2] += L::cz[i] * v;
      }
      const double rho = P.rho0 + d;
      const double w = peskin(cx - X[0]) * peskin(cy - X[1]) * peskin(cz - X[2]);
      for (int a = 0; a < 3; a++) U[a] = w * (j[a] + 0.5 * force[3 * node + a]) / rho;
    }
  }
  for (int o = 32; o > 0; o >>= 1)
    for (int a = 0; a < 3; a++) U[a] += __shfl_xor(U[a], o, 64);
  if (live && k == 0)
    for (int a = 0; a < 3; a++) {
      md.U[3 * g + a] = U[a];
      md.X[3 * g + a] = X[a] + U[a];
    }
}

// ---------------------------------------------------------------------------
// initial equilibria (3D) from staged fields: rho, phi, psi, ux, uy, uz
template <class St, typename R>
__global__ void k_init3d(St dst, LBParams P, const double* __restrict__ st,
                         const int* __restrict__ tflag, const int* __restrict__ tstate,
                         const double* __restrict__ Ifield) {
  using L = Lattice<19>;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
  double lap[3], ctr[3];
  for (int f = 0; f < 3; f++) {
    const double* F = st + (long long)f * P.N;
    ctr[f] = F[n];
    double acc = 0.0;
    for (int i = 1; i < 19; i++) {
      const long long nb = ((long long)fd_row(z + L::cz[i], P.nz, P.wall_z) * P.ny +
                            fd_row(y + L::cy[i], P.ny, P.wall_y)) * P.nx + wrap(x + L::cx[i], P.nx);
      acc += L::w(i) * (F[nb] - ctr[f]);
    }
    lap[f] = 6.0 * acc;
  }
  double I = 0.0;
  if (tflag[tile3(P, x, y, z)] == tstate[1]) I = Ifield[n];
  double mr, mp, ms;
  chem_pot(P, ctr[0] - P.rho0, ctr[1], ctr[2], lap[0], lap[1], lap[2], I, mr, mp, ms);
  const double u[3] = {st[3 * P.N + n], st[4 * P.N + n], st[5 * P.N + n]};
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double sp = -(P.psh[0] * ctr[1] + P.psh[1] * ctr[2]);  // lattice-pressure shift
  double E[3][19], gs = 0, hs = 0;
  for (int i = 0; i < 19; i++) {
    const double cu = L::cx[i] * u[0] + L::cy[i] * u[1] + L::cz[i] * u[2];
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
      for (int i = 1; i < 19; i++) {
        const double q = (double)dst.quantize((R)E[s][i]);
        E[s][0] += E[s][i] - q;
        E[s][i] = q;
      }
  }
  for (int i = 0; i < 19; i++) {
    const int sy = y - L::cy[i], sz = z - L::cz[i];
    long long tn;
    int dir = i;
    if ((P.wall_y && (sy < 0 || sy >= P.ny)) || (P.wall_z && (sz < 0 || sz >= P.nz))) {
      tn = n;
      dir = L::opp[i];
    } else {
      tn = ((long long)wrap(sz, P.nz) * P.ny + wrap(sy, P.ny)) * P.nx + wrap(x - L::cx[i], P.nx);
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

// moments readout (3D): out = [rho, C1, C2, C3, ux, uy, uz] x N
template <class St, typename R>
__global__ void k_moments3d(St cur, LBParams P, double* __restrict__ out) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P.N) return;
  const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
  R pf[19], pg[19], ph[19];
  double g0, h0, d, jx, jy, jz, phi, psi;
  pull19(cur, P, x, y, z, pf, pg, ph, g0, h0);
  moments19(pf, pg, ph, g0, h0, d, jx, jy, jz, phi, psi);
  const double rho = P.rho0 + d;
  double C[3];
  conc3(P, rho, phi, psi, C);
  out[n] = rho;
  out[P.N + n] = C[0];
  out[2 * P.N + n] = C[1];
  out[3 * P.N + n] = C[2];
  out[4 * P.N + n] = jx / rho;
  out[5 * P.N + n] = jy / rho;
  out[6 * P.N + n] = jz / rho;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_energy_nodes3d(LBParams P, const double* __restrict__ mom,
                                                       const int* __restrict__ tflag,
                                                       const int* __restrict__ tstate,
                                                       const double* __restrict__ Ifield,
                                                       double* __restrict__ part) {
  using L = Lattice<19>;
  __shared__ double sh[NT / 64];
  const long long n = (long long)blockIdx.x * NT + threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (n < P.N) {
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    const double kap[3] = {P.k1, P.k2, P.k3};
    for (int m = 0; m < 3; m++) {
      const double* C = mom + (long long)(1 + m) * P.N;
      const double c = C[n];
      double g[3] = {0, 0, 0};
      for (int i = 1; i < 19; i++) {
        const long long nb = ((long long)fd_row(z + L::cz[i], P.nz, P.wall_z) * P.ny +
                              fd_row(y + L::cy[i], P.ny, P.wall_y)) * P.nx + wrap(x + L::cx[i], P.nx);
        g[0] += L::w(i) * L::cx[i] * C[nb];
        g[1] += L::w(i) * L::cy[i] * C[nb];
        g[2] += L::w(i) * L::cz[i] * C[nb];
      }
      v[m] = c;
      v[3] += 0.5 * kap[m] * c * c * (1.0 - c) * (1.0 - c);
      v[4] += 0.5 * P.a2 * kap[m] * 9.0 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    }
    double I = 0;
    if (tflag[tile3(P, x, y, z)] == tstate[1]) I = Ifield[n];
    const double psi = mom[3 * P.N + n];
    v[5] = 0.5 * P.kc * (psi - I) * (psi - I);
    const double rho = mom[n];
    const double u0 = mom[4 * P.N + n], u1 = mom[5 * P.N + n], u2 = mom[6 * P.N + n];
    v[6] = 0.5 * rho * (u0 * u0 + u1 * u1 + u2 * u2);
    if (P.dens) {  // ideal gas of the number density, c_s^2 M_b n ln n
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

}  // namespace lb
