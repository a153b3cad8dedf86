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
constexpr int COUP3_CHUNK = 1024;
constexpr int COUP3_KEEP = 2;

struct MeshDev {
  int* tri;       // 3 per triangle, marker ids
  int* toff;      // K+1 triangle offsets
  int* edge;      // 4 per edge: a, b, t1, t2
  double* erest;  // rest length per edge
  int* eoff;      // K+1 edge offsets
  int* tadj;      // 3 per triangle: the triangle across edge (v_k, v_k+1)
  int* vtoff;     // M+1: vertex -> incident triangles (CSR)
  int* vt;
  double* fn;     // 3 per triangle: unit face normal (area vector direction)
  double* vn;     // 3 per vertex: angle-weighted normal
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

// does the ray from p towards +x cross triangle (a, b, c)?  (strict inside
// of the triangle's projection onto the yz plane)
__device__ __forceinline__ int ray_tri(const double* p, const double* a, const double* b,
                                       const double* c) {
  const double e0 = (b[1] - a[1]) * (p[2] - a[2]) - (b[2] - a[2]) * (p[1] - a[1]);
  const double e1 = (c[1] - b[1]) * (p[2] - b[2]) - (c[2] - b[2]) * (p[1] - b[1]);
  const double e2 = (a[1] - c[1]) * (p[2] - c[2]) - (a[2] - c[2]) * (p[1] - c[1]);
  const bool pos = e0 > 0 && e1 > 0 && e2 > 0, neg = e0 < 0 && e1 < 0 && e2 < 0;
  if (!pos && !neg) return 0;
  const double s = e0 + e1 + e2;
  const double xs = (e1 * a[0] + e2 * b[0] + e0 * c[0]) / s;
  return xs > p[0];
}

struct Coup3Args {
  int nx, ny, nz, wall_y, wall_z;
  double alpha, kappa_c, r_cut;
  int want_force;
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
  for (int a = 0; a < 3; a++) {
    const double cm = 0.5 * (bx[a] + bx[3 + a]);
    g.pc[a] = near_img(ct[a], cm, dims[a], per[a]);
    g.pp[a] = near_img((double)xi[a], cm, dims[a], per[a]);
    if (g.pc[a] + hd < bx[a] - reach || g.pc[a] - hd > bx[3 + a] + reach) g.miss = true;
    if (g.pp[a] < bx[a] - reach || g.pp[a] > bx[3 + a] + reach) g.inbox = false;
    if (per[a]) {
      const int s0 = t0[a], s1 = min(t0[a] + TILE3 - 1, dims[a] - 1);
      if (near_img((double)s0, cm, dims[a], 1) - s0 != near_img((double)s1, cm, dims[a], 1) - s1)
        g.split = true;
    }
  }
  if (g.split) g.miss = false;
  return g;
}

template <class St, typename R, int NT>
__global__ __launch_bounds__(NT) void k_coupling3d(MemDev md, MeshDev mh, TileMap tm, Coup3Args ca,
                                                   double* __restrict__ Ifield, St cur) {
  __shared__ int s_cand[COUP3_CHUNK];
  __shared__ int s_cnt;
  __shared__ double s_red[NT / 64];
  __shared__ int b_tri[COUP3_KEEP][NT];
  __shared__ double b_w[COUP3_KEEP][3][NT];
  __shared__ double b_sd[COUP3_KEEP][NT];
  const int ntl = tm.tstate[0];
  const double reach = ca.r_cut + 1.0;
  const double hd = 0.5 * TILE3 * 1.7320508075688772;
  const int per[3] = {1, !ca.wall_y, !ca.wall_z};
  const int dims[3] = {ca.nx, ca.ny, ca.nz};
  for (int li = blockIdx.x; li < ntl; li += gridDim.x) {
    const int t = tm.tlist[li];
    const int tx = t % tm.ntx, ty = (t / tm.ntx) % tm.nty, tz = t / (tm.ntx * tm.nty);
    const int t0[3] = {tx * TILE3, ty * TILE3, tz * TILE3};
    const int lt = (int)threadIdx.x;
    const int xi[3] = {t0[0] + lt % TILE3, t0[1] + (lt / TILE3) % TILE3, t0[2] + lt / (TILE3 * TILE3)};
    const bool valid = xi[0] < ca.nx && xi[1] < ca.ny && xi[2] < ca.nz;
    const double ct[3] = {t0[0] + 0.5 * (TILE3 - 1), t0[1] + 0.5 * (TILE3 - 1), t0[2] + 0.5 * (TILE3 - 1)};
    double Itot = 0.0;
    int kept = 0;
    for (int m = 0; m < md.K; m++) {
      const TileGeo g = tile_geo(md.mbox + 8 * m, ct, xi, t0, dims, per, hd, reach, valid);
      if (g.miss) continue;  // uniform over the block
      const int t0m = mh.toff[m], nt = mh.toff[m + 1] - t0m;
      const int slot = kept++;
      double d2b = 1e300, wb[3] = {0, 0, 0};
      int tb = -1;
      bool far = false;  // the whole tile lies beyond r_cut: I from the ray parity
      int par = 0;
      if (!g.split) {
        double dmin = 1e300;
        int cr = 0;
        // ray parity of the tile centre, with the same tiny offset of the ray
        // in y and z that keeps it off edges and vertices
        const double pr[3] = {g.pc[0], g.pc[1] + 1.2345678e-7, g.pc[2] + 2.3456789e-7};
        for (int q = threadIdx.x; q < nt; q += NT) {
          const int* tv = mh.tri + 3 * (t0m + q);
          double w[3];
          dmin = fmin(dmin, tri_d2(g.pc, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], w));
          cr += ray_tri(pr, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2]);
        }
        dmin = sqrt(block_min<NT>(dmin, s_red));
        par = ((int)block_sum<NT>((double)cr, s_red)) & 1;
        far = dmin > ca.r_cut + hd;
        if (!far) {
          // every node's closest triangle lies within dmin + 2 hd of the centre
          const double cull = dmin + 2.0 * hd + 1e-6;
          for (int c0 = 0; c0 < nt; c0 += COUP3_CHUNK) {
            if (threadIdx.x == 0) s_cnt = 0;
            __syncthreads();
            for (int q = c0 + threadIdx.x; q < min(nt, c0 + COUP3_CHUNK); q += NT) {
              const int* tv = mh.tri + 3 * (t0m + q);
              double w[3];
              if (tri_d2(g.pc, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], w) <= cull * cull)
                s_cand[atomicAdd(&s_cnt, 1)] = q;
            }
            __syncthreads();
            const int nc = s_cnt;
            if (g.inbox)
              for (int q = 0; q < nc; q++) {
                const int tq = s_cand[q];
                const int* tv = mh.tri + 3 * (t0m + tq);
                double w[3];
                const double d2 = tri_d2(g.pp, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], w);
                if (d2 < d2b || (d2 == d2b && tq < tb)) {
                  d2b = d2;
                  tb = tq;
                  wb[0] = w[0];
                  wb[1] = w[1];
                  wb[2] = w[2];
                }
              }
            __syncthreads();
          }
        }
      } else if (g.inbox) {
        // nodes of different images: each searches the whole mesh
        for (int q = 0; q < nt; q++) {
          const int* tv = mh.tri + 3 * (t0m + q);
          double w[3];
          const double d2 = tri_d2(g.pp, md.X + 3 * tv[0], md.X + 3 * tv[1], md.X + 3 * tv[2], w);
          if (d2 < d2b) {
            d2b = d2;
            tb = q;
            wb[0] = w[0];
            wb[1] = w[1];
            wb[2] = w[2];
          }
        }
      }
      double sd = 0.0;
      bool band = false;
      if (far) {
        if (g.inbox && par) Itot += 1.0;
      } else if (g.inbox && tb >= 0) {
        const int tg = t0m + tb;
        const int* tv = mh.tri + 3 * tg;
        double Qp[3] = {0, 0, 0}, nrm[3];
        for (int k = 0; k < 3; k++)
          for (int a = 0; a < 3; a++) Qp[a] += wb[k] * md.X[3 * tv[k] + a];
        const int zeros = (wb[0] == 0.0) + (wb[1] == 0.0) + (wb[2] == 0.0);
        if (zeros == 0) {
          for (int a = 0; a < 3; a++) nrm[a] = mh.fn[3 * tg + a];
        } else if (zeros == 1) {
          const int k = wb[0] == 0.0 ? 0 : (wb[1] == 0.0 ? 1 : 2);  // edge opposite vertex k
          const int nb = mh.tadj[3 * tg + (k + 1) % 3];
          for (int a = 0; a < 3; a++) nrm[a] = mh.fn[3 * tg + a] + mh.fn[3 * nb + a];
        } else {
          const int k = wb[0] != 0.0 ? 0 : (wb[1] != 0.0 ? 1 : 2);
          for (int a = 0; a < 3; a++) nrm[a] = mh.vn[3 * tv[k] + a];
        }
        double dv[3];
        sub3(g.pp, Qp, dv);
        const double o = md.mbox[8 * m + 6];
        const bool in = o * dot3d(dv, nrm) < 0.0;  // outward normals for o = +1
        const double d = sqrt(d2b);
        sd = in ? d : -d;
        band = d <= ca.r_cut;
        Itot += band ? 0.5 * (1.0 + tanh(sd / (2.0 * ca.alpha))) : (in ? 1.0 : 0.0);
      }
      if (slot < COUP3_KEEP) {
        b_tri[slot][threadIdx.x] = band ? t0m + tb : -1;
        b_w[slot][0][threadIdx.x] = wb[0];
        b_w[slot][1][threadIdx.x] = wb[1];
        b_w[slot][2][threadIdx.x] = wb[2];
        b_sd[slot][threadIdx.x] = sd;
      }
    }
    const long long node = valid ? ((long long)xi[2] * ca.ny + xi[1]) * ca.nx + xi[0] : 0;
    if (valid) Ifield[node] = Itot;
    if (ca.want_force) {
      if (kept > COUP3_KEEP && threadIdx.x == 0) md.status[1] = 1;
      double psi = 0.0;
      if (valid) {
        using L = Lattice<19>;
        psi = cur.rest(2, node);
        for (int i = 1; i < 19; i++) {
          const int sy = xi[1] - L::cy[i], sz = xi[2] - L::cz[i];
          long long sn;
          int dir = i;
          if ((ca.wall_y && (sy < 0 || sy >= ca.ny)) || (ca.wall_z && (sz < 0 || sz >= ca.nz))) {
            sn = node;
            dir = L::opp[i];
          } else {
            sn = ((long long)wrap(sz, ca.nz) * ca.ny + wrap(sy, ca.ny)) * ca.nx + wrap(xi[0] - L::cx[i], ca.nx);
          }
          psi += (double)cur.template load<R>(2, dir, sn);
        }
      }
      int slot = 0;
      for (int m = 0; m < md.K && slot < COUP3_KEEP; m++) {
        const TileGeo g = tile_geo(md.mbox + 8 * m, ct, xi, t0, dims, per, hd, reach, valid);
        if (g.miss) continue;
        const int my = slot++;
        const int tg = b_tri[my][threadIdx.x];
        if (tg < 0) continue;
        const double sd = b_sd[my][threadIdx.x];
        const double d = fabs(sd);
        if (d == 0.0) continue;
        const double w[3] = {b_w[my][0][threadIdx.x], b_w[my][1][threadIdx.x], b_w[my][2][threadIdx.x]};
        const int* tv = mh.tri + 3 * tg;
        double Qp[3] = {0, 0, 0};
        for (int k = 0; k < 3; k++)
          for (int a = 0; a < 3; a++) Qp[a] += w[k] * md.X[3 * tv[k] + a];
        const double sg = sd > 0.0 ? 1.0 : -1.0;
        const double ch = cosh(sd / (2.0 * ca.alpha));
        const double wgt = ca.kappa_c / (4.0 * ca.alpha) * (psi - Itot) / (ch * ch);
        for (int k = 0; k < 3; k++) {
          long long* A = md.Facc + 3 * tv[k];
          for (int a = 0; a < 3; a++) {
            const double gk = -sg * (g.pp[a] - Qp[a]) / d * wgt * w[k];
            atomicAdd((unsigned long long*)&A[a], (unsigned long long)to_fix(gk));
          }
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
  // spring: E = ks/2 (l/l0 - 1)^2 l0
  double dvec[3];
  sub3(pb, pa, dvec);
  const double len = sqrt(dot3d(dvec, dvec));
  const double s = ks * (len / mh.erest[e] - 1.0) / len;
  double fb[3] = {-s * dvec[0], -s * dvec[1], -s * dvec[2]};
  double fa[3] = {-fb[0], -fb[1], -fb[2]};
  acc_force(md.Facc, a, fa);
  acc_force(md.Facc, b, fb);
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
  double dvec[3];
  sub3(md.X + 3 * b, md.X + 3 * a, dvec);
  const double len = sqrt(dot3d(dvec, dvec));
  const double st = len / mh.erest[e] - 1.0;
  out[2 * e] = 0.5 * md.ks[m] * st * st * mh.erest[e];
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
      double d = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < 19; i++) {
        const int sy = yw - L::cy[i], sz = zw - L::cz[i];
        long long sn;
        int dir = i;
        if ((P.wall_y && (sy < 0 || sy >= P.ny)) || (P.wall_z && (sz < 0 || sz >= P.nz))) {
          sn = node;
          dir = L::opp[i];
        } else {
          sn = ((long long)wrap(sz, P.nz) * P.ny + wrap(sy, P.ny)) * P.nx + wrap(xw - L::cx[i], P.nx);
        }
        const double v = (double)cur.template load<R>(0, dir, sn);
        d += v;
        j[0] += L::cx[i] * v;
        j[1] += L::cy[i] * v;
        j[2] += L::cz[i] * v;
      }
      const double rho = 1.0 + d;
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
  chem_pot(P, ctr[0] - 1.0, ctr[1], ctr[2], lap[0], lap[1], lap[2], I, mr, mp, ms);
  const double u[3] = {st[3 * P.N + n], st[4 * P.N + n], st[5 * P.N + n]};
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double E[3][19], gs = 0, hs = 0;
  for (int i = 0; i < 19; i++) {
    const double cu = L::cx[i] * u[0] + L::cy[i] * u[1] + L::cz[i] * u[2];
    const double pu = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
    E[0][i] = L::w(i) * ((ctr[0] - 1.0) + ctr[0] * pu);
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
  const double rho = 1.0 + d;
  out[n] = rho;
  out[P.N + n] = 0.5 * (rho + phi - psi);
  out[2 * P.N + n] = 0.5 * (rho - phi - psi);
  out[3 * P.N + n] = psi;
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
    v[7] = rho * log(rho) / 3.0;
  }
  for (int k = 0; k < 8; k++) {
    const double s = block_sum<NT>(v[k], sh);
    if (threadIdx.x == 0) part[(long long)blockIdx.x * 8 + k] = s;
  }
}

}  // namespace lb
