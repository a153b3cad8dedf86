// lbib.hip -- host runtime and C ABI of the gfx950 ternary LB + IBM library.
//
// A simulation is an Engine<Store, Real> living inside the caller's device
// workspace.  The runtime carves the workspace, validates inputs, uploads
// membranes and initial fields, and enqueues the per-step kernel sequence
// (Sec. 3.3 ordering):
//   k_tiles       bounding boxes of the membranes at X(t), active-tile map
//   k_coupling    coupling profile I(X(t)) and coupling forces (needs psi(t))
//   k_memforce    strain + bending + coupling force per marker (FP64)
//   k_spread      marker forces onto the lattice (fixed-point atomics)
//   k_lb          fused pull-stream / moments / mu / force / collide
//   k_interp      v at t+1 interpolated at X(t), Euler update X(t+1)
// D3Q19 runs the same sequence with triangle meshes (face and vertex normals
// before the coupling, per-edge membrane forces) and a two-kernel lattice
// update (moment field, then the z-marching collide kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbib.h"
#include "common.h"
#include "k_ibm.h"
#include "k_ibm3d.h"
#include "k_lb.h"
#include "k_lb3d.h"
#include "k_misc.h"
#include "store.h"
#include "batch.h"
#include "k_mlp.h"

using namespace lb;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  char* base;
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

#define HIPCHK(call)                         \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return LBIB_EHIP;  \
  } while (0)

struct Layout {
  size_t pops[2];       // population buffers A, B
  size_t pop_bytes;     // bytes of one buffer
  size_t Ifield, fib, force, tflag, tlist, tstate, stage, part;
  size_t X, U, F, Facc, rest, moff, mid, ks, kb, law, mbox, status, memE, stab, sinv;
  // 2D coupling cache: per node and cached membrane slot, key and bound
  size_t ckey, clb;
  // 3D: moment field and triangle meshes
  size_t mom, tri, toff, edge, erest, eoff, emem, tadj, tedge, vtoff, vt, fn, vn, ttab, ctab, coff;
  int maxCl;
  int maxT, maxE;
  size_t total;
  long long ntiles;
  int ntx, nty, ntz, tile;
};

long long pop_bytes_per_node(int Q, int storage) {
  switch (storage) {
    case LBIB_FP32: return (3LL * Q - 2) * 4 + 2 * 8;  // FP32 with FP64 g_0, h_0
    case LBIB_FP64: return 3LL * Q * 8;
    default: return 3LL * (Q - 1) * 2 + 4 + 2 * 8;     // 16-bit moving, FP32 f_0, FP64 g_0, h_0
  }
}

int validate(const lbib_params* p) {
  if (!p) return LBIB_EINVAL;
  if (p->lattice != LBIB_D2Q9 && p->lattice != LBIB_D3Q19) return LBIB_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBIB_EINVAL;
  if (p->lattice == LBIB_D2Q9 && p->nz != 1) return LBIB_EINVAL;
  if (p->wall_y && p->ny < 2) return LBIB_EINVAL;
  if (p->lattice == LBIB_D3Q19 && p->wall_z && p->nz < 2) return LBIB_EINVAL;
  if (!(p->tau > 0.5) || !(p->tau_phi > 0.5) || !(p->tau_psi > 0.5)) return LBIB_EINVAL;
  if (!(p->alpha > 0.0) || !(p->kappa_c >= 0.0)) return LBIB_EINVAL;
  if (p->storage < 0 || p->storage > 3) return LBIB_EINVAL;
  if (p->max_markers < 0 || p->max_elems < 0 || p->max_membranes < 0) return LBIB_EINVAL;
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N > (1LL << 40)) return LBIB_EINVAL;
  if (p->lattice == LBIB_D3Q19 && p->nz > 65535) return LBIB_EINVAL;
  // the FP32 format addresses its planes through 32-bit buffer offsets
  const int Q = p->lattice == LBIB_D2Q9 ? 9 : 19;
  if (p->storage == LBIB_FP32 && ((3LL * Q - 2) * N * 4 > 0xffffffffLL || 2 * N * 8 > 0xffffffffLL))
    return LBIB_EINVAL;
  if (p->max_elems > (1 << 28) || p->max_markers > (1 << 28)) return LBIB_EINVAL;
  return LBIB_OK;
}

Layout make_layout(const lbib_params* p) {
  Layout L{};
  const int Q = p->lattice == LBIB_D2Q9 ? 9 : 19;
  const int D = p->lattice == LBIB_D2Q9 ? 2 : 3;
  const long long N = (long long)p->nx * p->ny * p->nz;
  static_assert((TILE2 & (TILE2 - 1)) == 0, "the lattice kernels index tiles by shifts");
  L.tile = D == 2 ? TILE2 : 8;
  L.ntx = (p->nx + L.tile - 1) / L.tile;
  L.nty = (p->ny + L.tile - 1) / L.tile;
  L.ntz = D == 3 ? (p->nz + L.tile - 1) / L.tile : 1;
  L.ntiles = (long long)L.ntx * L.nty * L.ntz;
  const int M = std::max(p->max_markers, 1), K = std::max(p->max_membranes, 1);
  Carver c{nullptr};
  L.pop_bytes = (size_t)(pop_bytes_per_node(Q, p->storage) * N);
  // 16-bit storage keeps the rest planes behind the moving planes
  L.pops[0] = c.take(L.pop_bytes + 2 * kAlign);
  L.pops[1] = c.take(L.pop_bytes + 2 * kAlign);
  L.Ifield = c.take((size_t)N * 8);
  L.fib = c.take((size_t)N * D * 8);
  L.force = c.take((size_t)N * D * 8);
  L.tflag = c.take((size_t)L.ntiles * 4);
  L.tlist = c.take((size_t)L.ntiles * 4);
  L.tstate = c.take(64);
  L.stage = c.take((size_t)N * 8 * 8);
  L.maxT = D == 3 ? std::max(p->max_elems, 1) : 0;
  L.maxE = 2 * L.maxT;  // a closed mesh has 3T/2 edges
  L.part = c.take((size_t)((N + 255) / 256 + 1) * 8 * 8 + (size_t)std::max(M, L.maxE) * 2 * 8);
  L.X = c.take((size_t)M * 3 * 8);
  L.U = c.take((size_t)M * 3 * 8);
  L.F = c.take((size_t)M * 3 * 8);
  L.Facc = c.take((size_t)M * 3 * 8);
  L.rest = c.take((size_t)M * 8);
  L.moff = c.take((size_t)(K + 1) * 4);
  L.mid = c.take((size_t)M * 4);
  L.ks = c.take((size_t)K * 8);
  L.kb = c.take((size_t)K * 8);
  L.law = c.take((size_t)K * 4);
  L.mbox = c.take((size_t)K * 8 * 8);
  L.status = c.take(64);
  L.memE = c.take(64);
  L.stab = c.take(D == 2 ? (size_t)M * 16 : 0);
  L.sinv = c.take(D == 2 ? (size_t)M * 4 : 0);
  L.ckey = c.take((size_t)(D == 2 ? COUP_CACHE : COUP3_CACHE) * N * 4);
  L.clb = c.take((size_t)(D == 2 ? COUP_CACHE : COUP3_CACHE) * N * 4);
  const bool d3 = D == 3;
  L.mom = c.take(d3 ? (size_t)N * 3 * 8 : 0);
  L.tri = c.take((size_t)L.maxT * 3 * 4);
  L.toff = c.take(d3 ? (size_t)(K + 1) * 4 : 0);
  L.edge = c.take((size_t)L.maxE * 4 * 4);
  L.erest = c.take((size_t)L.maxE * 8);
  L.eoff = c.take(d3 ? (size_t)(K + 1) * 4 : 0);
  L.emem = c.take((size_t)L.maxE * 4);
  L.tadj = c.take((size_t)L.maxT * 3 * 4);
  L.tedge = c.take((size_t)L.maxT * 3 * 4);
  L.vtoff = c.take(d3 ? (size_t)(M + 1) * 4 : 0);
  L.vt = c.take((size_t)L.maxT * 3 * 4);
  L.fn = c.take((size_t)L.maxT * 3 * 8);
  L.vn = c.take(d3 ? (size_t)M * 3 * 8 : 0);
  L.ttab = c.take((size_t)L.maxT * 4 * 16);
  L.maxCl = d3 ? L.maxT / CL3 + K : 0;  // 64-triangle clusters, one partial per mesh
  L.ctab = c.take((size_t)L.maxCl * 16);
  L.coff = c.take(d3 ? (size_t)(K + 1) * 4 : 0);
  L.total = c.off;
  return L;
}

}  // namespace

// ---------------------------------------------------------------------------
struct lbib_sim {
  lbib_params p{};
  Layout L{};
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int Q = 9, D = 2;
  long long N = 0;
  int cur = 0;  // index of the buffer holding the current state
  bool ready = false;
  long long steps = 0;
  int K = 0, M = 0;
  std::vector<int> moff{0};
  int ntri = 0, nedge = 0;                 // triangles and edges of all meshes (3D)
  std::vector<int> toff{0}, eoff{0}, vtoff{0}, coff{0};
  double r_cut = 0;
  int bx = 256, seg = 0;  // fused-kernel launch shape (seg 0: automatic)
  int tx3 = 32;           // D3Q19: x extent of the lattice kernel's 256-node tile (16, 32, 64)
  int nxcd = 0;           // L2 domains workgroups are dealt to (0: automatic, 1: plain order)
  int ring = 3;           // rows in the fused kernel's register ring (4: prefetch)
  int overlap = 0;        // 2D: lattice regions away from the membranes beside the
                          // membrane kernels (0 off, 1 on)
  int force_form = 0;     // force of eq. ForceFE, 0 potential form, 1 divergence form (D2Q9, the default there)
  int coup_cache = 1;     // each node keeps its closest membrane segment / triangle between steps
  double fext[3] = {0, 0, 0};  // uniform external force density (eq. ForcingTermLBE)
  double mw[3] = {1, 1, 1};    // component densities (eq. MassDensity)
  bool any_law = false;   // D3Q19: a mesh has a triangle strain law (the triangle pass runs)
  lbib_sim* owner = nullptr;  // the batch this simulation belongs to (it owns the handle)
  // optional per-phase timing with HIP events on the stream
  int timing = 0;  // bit mask of timed phases
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;
  size_t ev_used = 0;
  int timed_steps = 0;
  double timed_ms[4] = {0, 0, 0, 0};
  hipEvent_t ev() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  // begin a timed phase on stream s (default: the simulation's stream):
  // returns the start event (or null when not timing)
  hipEvent_t tbeg(int phase, hipStream_t s = nullptr) {
    if (!(timing >> phase & 1)) return nullptr;
    hipEvent_t e = ev();
    if (e) (void)hipEventRecord(e, s ? s : stream);
    return e;
  }
  void tend(int phase, hipEvent_t start, hipStream_t s = nullptr) {
    if (!start) return;
    hipEvent_t e = ev();
    if (!e) return;
    (void)hipEventRecord(e, s ? s : stream);
    ev_open.push_back({phase, {start, e}});
  }
  int timing_flush() {
    if (ev_open.empty()) return LBIB_OK;
    if (hipStreamSynchronize(stream) != hipSuccess) return LBIB_EHIP;
    for (auto& q : ev_open) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, q.second.first, q.second.second) != hipSuccess) return LBIB_EHIP;
      timed_ms[q.first] += ms;
    }
    ev_open.clear();
    ev_used = 0;
    return LBIB_OK;
  }
  virtual ~lbib_sim() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
  }
  virtual void setup() = 0;
  virtual int init(const double* stage_dev) = 0;
  virtual int step() = 0;
  virtual int moments(double* out_dev) = 0;
  virtual int energy_nodes(double* part, long long* nblk) = 0;
  virtual int coupling(int want_force) = 0;
  virtual int check(int* bad_dev) = 0;
  // per-element membrane energies (strain, bending) into out[2 * rows]
  virtual int mem_energy(double* out, long long* rows) = 0;
  // a member's membranes or state changed (a batch rebuilds its tables)
  virtual void mark_dirty() {}
  // forget every node's cached closest segment (markers moved other than by
  // a step: checkpoint load, marker poke)
  int drop_coupling_cache() {
    if (!L.ckey) return LBIB_OK;
    if (hipMemsetAsync(ws + L.ckey, 0xff, (size_t)(D == 2 ? COUP_CACHE : COUP3_CACHE) * N * 4, stream) !=
        hipSuccess)
      return LBIB_EHIP;
    return LBIB_OK;
  }
  virtual bool is_batch() const { return false; }
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  MemDev memdev() const {
    MemDev m;
    m.X = at<double>(L.X);
    m.U = at<double>(L.U);
    m.F = at<double>(L.F);
    m.Facc = at<long long>(L.Facc);
    m.rest = at<double>(L.rest);
    m.moff = at<int>(L.moff);
    m.mid = at<int>(L.mid);
    m.ks = at<double>(L.ks);
    m.kb = at<double>(L.kb);
    m.law = at<int>(L.law);
    m.mbox = at<double>(L.mbox);
    m.status = at<int>(L.status);
    m.stab = at<float4>(L.stab);
    m.sinv = at<float>(L.sinv);
    m.K = K;
    m.M = M;
    return m;
  }
  MeshDev meshdev() const {
    MeshDev h;
    h.tri = at<int>(L.tri);
    h.toff = at<int>(L.toff);
    h.edge = at<int>(L.edge);
    h.erest = at<double>(L.erest);
    h.eoff = at<int>(L.eoff);
    h.tadj = at<int>(L.tadj);
    h.vtoff = at<int>(L.vtoff);
    h.vt = at<int>(L.vt);
    h.fn = at<double>(L.fn);
    h.vn = at<double>(L.vn);
    h.coff = at<int>(L.coff);
    h.tedge = at<int>(L.tedge);
    h.T = ntri;
    h.E = nedge;
    return h;
  }
  TileMap tilemap() const {
    TileMap t;
    t.tflag = at<int>(L.tflag);
    t.tlist = at<int>(L.tlist);
    t.tstate = at<int>(L.tstate);
    t.ntx = L.ntx;
    t.nty = L.nty;
    t.ntz = L.ntz;
    t.tile = L.tile;
    return t;
  }
};

namespace {

template <class St>
St make_store(char* base, long long N);
template <>
PlainStore<float, 9> make_store<PlainStore<float, 9>>(char* base, long long N) {
  return PlainStore<float, 9>{reinterpret_cast<float*>(base), N};
}
template <>
MixStore<9> make_store<MixStore<9>>(char* base, long long N) {
  size_t fl = align_up((size_t)(MixStore<9>::float_planes() * N * 4));
  return MixStore<9>{reinterpret_cast<float*>(base), reinterpret_cast<double*>(base + fl), N};
}
template <>
PlainStore<double, 9> make_store<PlainStore<double, 9>>(char* base, long long N) {
  return PlainStore<double, 9>{reinterpret_cast<double*>(base), N};
}
template <>
Split16Store<__half, 9> make_store<Split16Store<__half, 9>>(char* base, long long N) {
  const size_t mov = align_up((size_t)(3LL * 8 * N * 2)), r0 = align_up((size_t)(N * 4));
  return Split16Store<__half, 9>{reinterpret_cast<__half*>(base), reinterpret_cast<float*>(base + mov),
                                  reinterpret_cast<double*>(base + mov + r0), N};
}
template <>
Split16Store<__hip_bfloat16, 9> make_store<Split16Store<__hip_bfloat16, 9>>(char* base, long long N) {
  const size_t mov = align_up((size_t)(3LL * 8 * N * 2)), r0 = align_up((size_t)(N * 4));
  return Split16Store<__hip_bfloat16, 9>{reinterpret_cast<__hip_bfloat16*>(base), reinterpret_cast<float*>(base + mov),
                                  reinterpret_cast<double*>(base + mov + r0), N};
}

template <>
MixStore<19> make_store<MixStore<19>>(char* base, long long N) {
  size_t fl = align_up((size_t)(MixStore<19>::float_planes() * N * 4));
  return MixStore<19>{reinterpret_cast<float*>(base), reinterpret_cast<double*>(base + fl), N};
}
template <>
PlainStore<double, 19> make_store<PlainStore<double, 19>>(char* base, long long N) {
  return PlainStore<double, 19>{reinterpret_cast<double*>(base), N};
}
template <>
Split16Store<__half, 19> make_store<Split16Store<__half, 19>>(char* base, long long N) {
  const size_t mov = align_up((size_t)(3LL * 18 * N * 2)), r0 = align_up((size_t)(N * 4));
  return Split16Store<__half, 19>{reinterpret_cast<__half*>(base), reinterpret_cast<float*>(base + mov),
                                  reinterpret_cast<double*>(base + mov + r0), N};
}
template <>
Split16Store<__hip_bfloat16, 19> make_store<Split16Store<__hip_bfloat16, 19>>(char* base, long long N) {
  const size_t mov = align_up((size_t)(3LL * 18 * N * 2)), r0 = align_up((size_t)(N * 4));
  return Split16Store<__hip_bfloat16, 19>{reinterpret_cast<__hip_bfloat16*>(base), reinterpret_cast<float*>(base + mov),
                                  reinterpret_cast<double*>(base + mov + r0), N};
}

// lattice parameters shared by both engines
// The concentrations as a linear map of (rho, phi, psi) for component
// densities M_m (eq. MassDensity with eq. VariableTransform): with
// M_b = (M_1 + M_2)/2 and a = (M_1 - M_2)/2, the mass density is
// rho = M_b (C_1 + C_2) + a phi + M_3 psi, so C_1 + C_2 = (rho - a phi - M_3 psi)/M_b
// and C_{1,2} = ((C_1 + C_2) +- phi)/2.  The lattice's pressure is the ideal
// gas of the number density n = sum_m C_m, c_s^2 M_b n = c_s^2 (rho - a phi - b psi)
// with b = M_3 - M_b.
void density_map(LBParams& P, const double* mw) {
  const double mb = 0.5 * (mw[0] + mw[1]), a = 0.5 * (mw[0] - mw[1]), b = mw[2] - mb;
  const double s[3] = {1.0 / mb, -a / mb, -mw[2] / mb};  // C_1 + C_2 per unit of rho, phi, psi
  for (int q = 0; q < 3; q++) {
    P.cm[0][q] = 0.5 * (s[q] + (q == 1 ? 1.0 : 0.0));
    P.cm[1][q] = 0.5 * (s[q] - (q == 1 ? 1.0 : 0.0));
    P.cm[2][q] = q == 2 ? 1.0 : 0.0;
  }
  P.psh[0] = a;
  P.psh[1] = b;
  P.mb = mb;
  P.rho0 = mb;
  P.dens = (mw[0] != 1.0 || mw[1] != 1.0 || mw[2] != 1.0) ? 1 : 0;
}

void fill_params(LBParams& P, const lbib_params& p, const Layout& L, long long N, int seg, const double* fext,
                 const double* mw) {
  P.inv_tau = (1.0 / p.tau);
  P.inv_tau_phi = (1.0 / p.tau_phi);
  P.inv_tau_psi = (1.0 / p.tau_psi);
  P.gphi = p.gamma_phi;
  P.gpsi = p.gamma_psi;
  P.k1 = p.kappa[0];
  P.k2 = p.kappa[1];
  P.k3 = p.kappa[2];
  P.a2 = p.alpha * p.alpha;
  P.kc = p.kappa_c;
  for (int a = 0; a < 3; a++) P.fext[a] = fext[a];
  density_map(P, mw);
  P.nx = p.nx;
  P.ny = p.ny;
  P.nz = p.lattice == LBIB_D3Q19 ? p.nz : 1;
  P.wall_y = p.wall_y;
  P.wall_z = p.lattice == LBIB_D3Q19 ? p.wall_z : 0;
  P.N = N;
  P.ntx = L.ntx;
  P.nty = L.nty;
  P.tile = L.tile;
  P.seg = seg;
  P.mode = 0;
  P.seg2 = 0;
  P.npiece = 1;
}

template <class St, typename R>
struct Engine2D final : lbib_sim {
  LBParams P{};
  St store(int which) const { return make_store<St>(ws + L.pops[which], N); }

  void setup() override { fill_params(P, p, L, N, seg, fext, mw); }

  CoupArgs coup_args(int want_force) const {
    CoupArgs c;
    c.nx = p.nx;
    c.ny = p.ny;
    c.wall_y = p.wall_y;
    c.alpha = p.alpha;
    c.kappa_c = p.kappa_c;
    c.r_cut = r_cut;
    c.want_force = want_force;
    c.ckey = coup_cache ? at<int>(L.ckey) : nullptr;
    c.clb = coup_cache ? at<float>(L.clb) : nullptr;
    c.N = N;
    return c;
  }

  // stamp of the last tile pass: the host chooses it for a simulation of its
  // own (one launch fewer per step); a batch member's stamps advance on the
  // device with its batch, so it keeps the begin kernel
  int tile_stamp = 1;
  // the counter holding the last tile pass's active-tile count
  const int* tile_count() const { return at<int>(L.tstate) + (owner ? 0 : 4 + (tile_stamp & 1)); }
  // boxes, segment table and active-tile map at X(t)
  void tiles_pass() {
    MemDev md = memdev();
    TileMap tm = tilemap();
    int stamp = 0;
    if (owner)
      hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, stream, tm.tstate);
    else
      stamp = ++tile_stamp;
    hipLaunchKernelGGL(k_tiles<256>, dim3(K), dim3(256), 0, stream, md, tm, p.nx, p.ny, 1, p.wall_y,
                       0, 2, map_reach(r_cut), stamp);
  }
  // profile field and coupling forces on the active tiles
  void profile_pass(int want_force) {
    const int grid = (int)std::min<long long>(std::max<long long>(L.ntiles, 1), 2048);
    hipLaunchKernelGGL((k_coupling2d<St, R, COUP_THREADS>), dim3(grid), dim3(COUP_THREADS), 0, stream,
                       memdev(), tilemap(), coup_args(want_force), at<double>(L.Ifield), store(cur),
                       tile_count());
  }
  int coupling(int want_force) override {
    if (K == 0) return LBIB_OK;
    tiles_pass();
    profile_pass(want_force);
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  // second stream and events of the overlapped step (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int ensure_side() {
    if (side) return LBIB_OK;
    if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) {
      side = nullptr;
      return LBIB_EHIP;
    }
    if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess)
      return LBIB_EHIP;
    return LBIB_OK;
  }
  ~Engine2D() override {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
  }
  // overlap the lattice regions away from the membranes with the membrane
  // kernels?  Only on request: the two lattice passes then share the memory
  // bandwidth with each other and with the membrane kernels
  bool split_step() const { return K > 0 && overlap > 0; }

  // kernel variant for the current (bx, ring, force form)
  template <int WPE3, int FORM>
  const void* lb_kernel_f() const {
    if (ring == 4) {
      if (bx == 128) return (const void*)&k_lb2d<St, R, 128, 4, 2, FORM>;
      if (bx == 192) return (const void*)&k_lb2d<St, R, 192, 4, 2, FORM>;
      if (bx == 256) return (const void*)&k_lb2d<St, R, 256, 4, 2, FORM>;
      return (const void*)&k_lb2d<St, R, 64, 4, 2, FORM>;
    }
    if (bx == 128) return (const void*)&k_lb2d<St, R, 128, 3, WPE3, FORM>;
    if (bx == 192) return (const void*)&k_lb2d<St, R, 192, 3, WPE3, FORM>;
    if (bx == 256) return (const void*)&k_lb2d<St, R, 256, 3, WPE3, FORM>;
    return (const void*)&k_lb2d<St, R, 64, 3, WPE3, FORM>;
  }
  // the divergence form keeps three more fields in LDS, which leaves room
  // for two waves per SIMD: its register budget is sized for that
  const void* lb_kernel() const { return force_form ? lb_kernel_f<2, 1>() : lb_kernel_f<3, 0>(); }

  // rows per workgroup: with seg = 0 (automatic), the whole lattice is cut
  // into exactly as many (strip, segment) workgroups as can be resident at
  // once, so no partial last round of workgroups stretches the launch
  int pick_seg() const {
    if (seg > 0) return seg;
    const int W = bx - 4;
    const long long nstrip = (p.nx + W - 1) / W;
    int per_cu = 0, ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lb_kernel(), bx, 0) != hipSuccess ||
        per_cu <= 0 || ncu <= 0)
      return std::max(4, std::min(p.ny, 16));
    const long long slots = (long long)per_cu * ncu;
    long long rows = std::max(4LL, std::min<long long>(p.ny, (p.ny * nstrip + slots - 1) / slots));
    // rounding the segment count up can still leave a few workgroups over
    while (rows < p.ny && nstrip * ((p.ny + rows - 1) / rows) > slots) rows++;
    return (int)rows;
  }

  // the fused kernel on stream s over the whole lattice (mode 0), the
  // regions that read no membrane field (1) or the others in pieces (2)
  void launch_lb(St src, St dst, hipStream_t s, int mode) {
    P.seg = pick_seg();
    const int W = bx - 4;
    P.nstrip = (p.nx + W - 1) / W;
    P.nseg = (p.ny + P.seg - 1) / P.seg;
    // automatic: eight L2 domains (the XCDs), so a segment's vertical
    // neighbours, which read the same halo rows at the same time, sit in
    // the same L2 (fetched bytes -15 % on the 2048^2 workload)
    P.nxcd = nxcd > 0 ? nxcd : 8;
    P.mode = mode;
    P.npiece = mode == 2 ? (P.seg + 5) / 6 : 1;  // pieces of about five rows
    P.seg2 = (P.seg + P.npiece - 1) / P.npiece;
    dim3 grid(P.nstrip * P.nseg * P.npiece);
    const int* tf = at<int>(L.tflag);
    const int* ts = at<int>(L.tstate);
    const double* If = at<double>(L.Ifield);
    long long* fib = at<long long>(L.fib);
    double* frc = at<double>(L.force);
    // (lanes, ring depth, waves per SIMD) variants of the fused kernel
#define LB_LAUNCH(BXV, NSV, WPEV)                                                                  \
  do {                                                                                             \
    if (mode == 0 && force_form == 1)                                                              \
      hipLaunchKernelGGL((k_lb2d<St, R, BXV, NSV, 2, 1>), grid, dim3(BXV), 0, s, src, dst, P, tf, ts, If, \
                         fib, frc);                                                                \
    else if (mode == 0)                                                                            \
      hipLaunchKernelGGL((k_lb2d<St, R, BXV, NSV, WPEV>), grid, dim3(BXV), 0, s, src, dst, P, tf, ts, If, \
                         fib, frc);                                                                \
    else if (force_form == 1)                                                                      \
      hipLaunchKernelGGL((k_lb2d_part<St, R, BXV, NSV, 2, 1>), grid, dim3(BXV), 0, s, src, dst, P, tf, ts, \
                         If, fib, frc);                                                            \
    else                                                                                           \
      hipLaunchKernelGGL((k_lb2d_part<St, R, BXV, NSV, WPEV>), grid, dim3(BXV), 0, s, src, dst, P, tf, ts, \
                         If, fib, frc);                                                            \
  } while (0)
    if (ring == 4) {
      if (bx == 128) LB_LAUNCH(128, 4, 2);
      else if (bx == 192) LB_LAUNCH(192, 4, 2);
      else if (bx == 256) LB_LAUNCH(256, 4, 2);
      else LB_LAUNCH(64, 4, 2);
    } else {
      if (bx == 128) LB_LAUNCH(128, 3, 3);
      else if (bx == 192) LB_LAUNCH(192, 3, 3);
      else if (bx == 256) LB_LAUNCH(256, 3, 3);
      else LB_LAUNCH(64, 3, 3);
    }
#undef LB_LAUNCH
  }

  int step() override {
    MemDev md = memdev();
    const int mb16 = (16 * M + 255) / 256;  // sixteen lanes per marker
    const bool split = split_step();
    if (split && ensure_side() != LBIB_OK) return LBIB_EHIP;
    if (K > 0) {
      hipEvent_t t0 = tbeg(1);
      tiles_pass();
      if (split) {
        // the regions away from the membranes need only the tile map: they
        // run on the second stream beside the profile and force kernels
        if (hipEventRecord(ev_fork, stream) != hipSuccess || hipStreamWaitEvent(side, ev_fork, 0) != hipSuccess)
          return LBIB_EHIP;
        hipEvent_t ta = tbeg(0, side);
        launch_lb(store(cur), store(1 - cur), side, 1);
        tend(0, ta, side);
        if (hipEventRecord(ev_join, side) != hipSuccess) return LBIB_EHIP;
      }
      profile_pass(1);
      tend(1, t0);
      t0 = tbeg(2);
      hipLaunchKernelGGL(k_forcespread2d, dim3(mb16), dim3(256), 0, stream, md, at<long long>(L.fib), p.nx,
                         p.ny, p.wall_y);
      tend(2, t0);
    }
    hipEvent_t t1 = tbeg(0);
    launch_lb(store(cur), store(1 - cur), stream, split ? 2 : 0);
    tend(0, t1);
    if (split && hipStreamWaitEvent(stream, ev_join, 0) != hipSuccess) return LBIB_EHIP;
    if (K > 0) {
      hipEvent_t t2 = tbeg(3);
      hipLaunchKernelGGL((k_interp2d<St, R>), dim3(mb16), dim3(256), 0, stream, md, store(1 - cur), P,
                         (const double*)at<double>(L.force));
      tend(3, t2);
    }
    cur = 1 - cur;
    if (timing) {
      timed_steps++;
      if (ev_used > 4096) {
        int rc = timing_flush();
        if (rc) return rc;
      }
    }
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int init(const double* st) override {
    int rc = coupling(0);
    if (rc) return rc;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_init2d<St, R>), dim3(nb), dim3(256), 0, stream, store(cur), P, st, st + N,
                       st + 2 * N, st + 3 * N, st + 4 * N, (const int*)at<int>(L.tflag),
                       (const int*)at<int>(L.tstate), (const double*)at<double>(L.Ifield));
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int moments(double* out) override {
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_moments2d<St, R>), dim3(nb), dim3(256), 0, stream, store(cur), P, out);
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int energy_nodes(double* part, long long* nblk) override {
    const long long nb = (N + 255) / 256;
    hipLaunchKernelGGL((k_energy_nodes2d<256>), dim3((unsigned)nb), dim3(256), 0, stream, P,
                       (const double*)at<double>(L.stage), (const int*)at<int>(L.tflag),
                       (const int*)at<int>(L.tstate), (const double*)at<double>(L.Ifield), part);
    *nblk = nb;
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int check(int* bad) override {
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_check<St, R, 256>), dim3(nb), dim3(256), 0, stream, store(cur), N, 9, bad);
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int mem_energy(double* out, long long* rows) override {
    hipLaunchKernelGGL(k_memenergy2d, dim3((M + 255) / 256), dim3(256), 0, stream, memdev(), out);
    *rows = M;
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }
};

// D3Q19 with closed triangle meshes
template <class St, typename R>
struct Engine3D final : lbib_sim {
  LBParams P{};
  St store(int which) const { return make_store<St>(ws + L.pops[which], N); }
  int ntilex() const { return (p.nx + tx3 - 1) / tx3; }
  int ntiley() const { return (p.ny + 256 / tx3 - 1) / (256 / tx3); }
  const void* lb3_kernel() const {
    if (tx3 == 32) return (const void*)&k_lb3d<St, R, 32>;
    if (tx3 == 64) return (const void*)&k_lb3d<St, R, 64>;
    return (const void*)&k_lb3d<St, R, 16>;
  }

  void setup() override { fill_params(P, p, L, N, seg, fext, mw); }

  Moments3 mom3() const {
    Moments3 m;
    m.d = at<double>(L.mom);
    m.phi = m.d + N;
    m.psi = m.d + 2 * N;
    return m;
  }

  Coup3Args coup_args(int want_force) const {
    Coup3Args c;
    c.nx = p.nx;
    c.ny = p.ny;
    c.nz = p.nz;
    c.wall_y = p.wall_y;
    c.wall_z = p.wall_z;
    c.alpha = p.alpha;
    c.kappa_c = p.kappa_c;
    c.r_cut = r_cut;
    c.want_force = want_force;
    c.ckey = coup_cache ? at<int>(L.ckey) : nullptr;
    c.clb = coup_cache ? at<float>(L.clb) : nullptr;
    c.N = N;
    return c;
  }

  // mesh geometry at X(t): boxes and the active-tile map, face normals,
  // orientation, vertex normals; then the profile and coupling forces
  int coupling(int want_force) override {
    if (K == 0) return LBIB_OK;
    MemDev md = memdev();
    MeshDev mh = meshdev();
    TileMap tm = tilemap();
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, stream, tm.tstate);
    hipLaunchKernelGGL(k_tiles<256>, dim3(K), dim3(256), 0, stream, md, tm, p.nx, p.ny, p.nz, p.wall_y,
                       p.wall_z, 3, map_reach(r_cut), 0);
    hipLaunchKernelGGL(k_facenormals, dim3((ntri + 255) / 256), dim3(256), 0, stream, md, mh);
    hipLaunchKernelGGL(k_meshvolume<256>, dim3(K), dim3(256), 0, stream, md, mh);
    hipLaunchKernelGGL(k_vertexnormals, dim3((M + 255) / 256), dim3(256), 0, stream, md, mh);
    hipLaunchKernelGGL(k_tritable3d, dim3((ntri + 255) / 256), dim3(256), 0, stream, md, mh, at<float4>(L.ttab));
    const int ncl = coff.back();
    hipLaunchKernelGGL(k_clusters3d, dim3((ncl * 64 + 255) / 256), dim3(256), 0, stream, md, mh,
                       (const float4*)at<float4>(L.ttab), at<float4>(L.ctab), ncl);
    // resident workgroups only: they take the active tiles from a counter
    const int grid = (int)std::min<long long>(std::max<long long>(L.ntiles, 1), coup3_slots());
    hipLaunchKernelGGL((k_coupling3d<St, R, COUP3_THREADS>), dim3(grid), dim3(COUP3_THREADS), 0, stream,
                       md, mh, tm, coup_args(want_force), (const float4*)at<float4>(L.ttab),
                       (const float4*)at<float4>(L.ctab), at<double>(L.Ifield), store(cur));
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  // workgroups of the profile kernel resident at once (queried once)
  int c3slots = 0;
  int coup3_slots() {
    if (c3slots > 0) return c3slots;
    int per_cu = 0, ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&k_coupling3d<St, R, COUP3_THREADS>,
                                                     COUP3_THREADS, 0) != hipSuccess ||
        per_cu <= 0 || ncu <= 0)
      return 1024;
    c3slots = per_cu * ncu;
    return c3slots;
  }

  // planes per workgroup: with seg = 0, one resident round of workgroups
  int pick_seg() const {
    if (seg > 0) return std::min(seg, p.nz);
    const long long tiles = (long long)ntilex() * ntiley();
    int per_cu = 0, ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lb3_kernel(), 256, 0) != hipSuccess ||
        per_cu <= 0 || ncu <= 0)
      return std::min(p.nz, 16);
    const long long slots = (long long)per_cu * ncu;
    const long long planes = (p.nz * tiles + slots - 1) / slots;
    return (int)std::max<long long>(std::min<long long>(4, p.nz), std::min<long long>(p.nz, planes));
  }

  void launch_lb(St src, St dst) {
    P.seg = pick_seg();
    P.nseg = (p.nz + P.seg - 1) / P.seg;
    P.nxcd = nxcd > 0 ? nxcd : 8;
    Moments3 m3 = mom3();
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_mom3d<St, R>), dim3(nb), dim3(256), 0, stream, src, P, m3);
    dim3 grid(ntilex() * ntiley(), P.nseg);
#define LB3_LAUNCH(TXV)                                                                             \
  hipLaunchKernelGGL((k_lb3d<St, R, TXV>), grid, dim3(256), 0, stream, src, dst, P, m3,             \
                     (const int*)at<int>(L.tflag), (const int*)at<int>(L.tstate),                   \
                     (const double*)at<double>(L.Ifield), at<long long>(L.fib), at<double>(L.force), \
                     ntilex())
    if (tx3 == 32)
      LB3_LAUNCH(32);
    else if (tx3 == 64)
      LB3_LAUNCH(64);
    else
      LB3_LAUNCH(16);
#undef LB3_LAUNCH
  }

  int step() override {
    MemDev md = memdev();
    MeshDev mh = meshdev();
    const int mb = (M + 255) / 256;
    const int mb64 = (int)((64LL * M + 255) / 256);  // one wave per marker
    if (K > 0) {
      hipEvent_t t0 = tbeg(1);
      int rc = coupling(1);
      if (rc) return rc;
      tend(1, t0);
      t0 = tbeg(2);
      hipLaunchKernelGGL(k_memedge3d, dim3((nedge + 255) / 256), dim3(256), 0, stream, md, mh,
                         (const int*)at<int>(L.emem));
      if (any_law)
        hipLaunchKernelGGL(k_memtri3d, dim3((ntri + 255) / 256), dim3(256), 0, stream, md, mh);
      hipLaunchKernelGGL(k_memforce3d, dim3(mb), dim3(256), 0, stream, md);
      hipLaunchKernelGGL(k_spread3d, dim3(mb64), dim3(256), 0, stream, md, at<long long>(L.fib), p.nx,
                         p.ny, p.nz, p.wall_y, p.wall_z);
      tend(2, t0);
    }
    hipEvent_t t1 = tbeg(0);
    launch_lb(store(cur), store(1 - cur));
    tend(0, t1);
    if (K > 0) {
      hipEvent_t t2 = tbeg(3);
      hipLaunchKernelGGL((k_interp3d<St, R>), dim3(mb64), dim3(256), 0, stream, md, store(1 - cur), P,
                         (const double*)at<double>(L.force));
      tend(3, t2);
    }
    cur = 1 - cur;
    if (timing) {
      timed_steps++;
      if (ev_used > 4096) {
        int rc = timing_flush();
        if (rc) return rc;
      }
    }
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int init(const double* st) override {
    int rc = coupling(0);
    if (rc) return rc;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_init3d<St, R>), dim3(nb), dim3(256), 0, stream, store(cur), P, st,
                       (const int*)at<int>(L.tflag), (const int*)at<int>(L.tstate),
                       (const double*)at<double>(L.Ifield));
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int moments(double* out) override {
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_moments3d<St, R>), dim3(nb), dim3(256), 0, stream, store(cur), P, out);
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int energy_nodes(double* part, long long* nblk) override {
    const long long nb = (N + 255) / 256;
    hipLaunchKernelGGL((k_energy_nodes3d<256>), dim3((unsigned)nb), dim3(256), 0, stream, P,
                       (const double*)at<double>(L.stage), (const int*)at<int>(L.tflag),
                       (const int*)at<int>(L.tstate), (const double*)at<double>(L.Ifield), part);
    *nblk = nb;
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int check(int* bad) override {
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL((k_check<St, R, 256>), dim3(nb), dim3(256), 0, stream, store(cur), N, 19, bad);
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }

  int mem_energy(double* out, long long* rows) override {
    MemDev md = memdev();
    MeshDev mh = meshdev();
    hipLaunchKernelGGL(k_facenormals, dim3((ntri + 255) / 256), dim3(256), 0, stream, md, mh);
    hipLaunchKernelGGL(k_memenergy3d, dim3((nedge + 255) / 256), dim3(256), 0, stream, md, mh,
                       (const int*)at<int>(L.emem), out);
    *rows = nedge;
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }
};


// Many D2Q9 simulations in one workspace, stepped together (FP32 storage).
// Members are ordinary simulations on their own slices of the workspace;
// the batch owns them.  Each phase of a step is one launch over all members
// (the lattice update one launch per size class), and the whole step is
// captured once per buffer parity in a hipGraph and replayed.
struct BatchEngine2D final : lbib_sim {
  using St = MixStore<9>;
  using R = float;
  using Mem = Engine2D<St, R>;
  std::vector<Mem*> mem;
  static constexpr int NCLS = 3;  // size classes by lattice width: <= 128, <= 256, larger
  int cls_bx[NCLS] = {64, 128, 256}, cls_seg[NCLS] = {0, 0, 0}, cls_ring[NCLS] = {3, 3, 3};
  bool use_graph = true, dirty = true, graph_ok = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  size_t off_tab = 0, off_mems = 0, off_mpre = 0, off_cm = 0, off_bpre = 0;
  int nmems = 0, Mtot = 0, cgrid = 1;
  int ncm[NCLS] = {0, 0, 0}, lgrid[NCLS] = {0, 0, 0}, lseg[NCLS] = {0, 0, 0};

  ~BatchEngine2D() override {
    drop_graphs();
    for (auto m : mem) delete m;
  }
  void drop_graphs() {
    for (auto& e : gexec)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
    graph_ok = false;
  }
  bool is_batch() const override { return true; }
  void mark_dirty() override { dirty = true; }
  void setup() override {}
  int init(const double*) override { return LBIB_ESTATE; }
  int moments(double*) override { return LBIB_ESTATE; }
  int energy_nodes(double*, long long*) override { return LBIB_ESTATE; }
  int coupling(int) override { return LBIB_ESTATE; }
  int check(int* bad) override {
    for (auto m : mem) {
      int rc = m->check(bad);
      if (rc) return rc;
    }
    return LBIB_OK;
  }
  int mem_energy(double*, long long*) override { return LBIB_ESTATE; }

  static int size_class(int nx) { return nx <= 128 ? 0 : (nx <= 256 ? 1 : 2); }
  static size_t table_bytes(int n, int kmax) {
    return align_up((size_t)n * sizeof(BMember<St>)) + align_up((size_t)std::max(kmax, 1) * sizeof(int2)) +
           align_up((size_t)(n + 1) * 4) + align_up((size_t)NCLS * n * 4) + align_up((size_t)NCLS * (n + 1) * 4);
  }
  template <int WPE3, int FORM>
  const void* lb_kernel_f(int c) const {
    const int bx = cls_bx[c];
    if (cls_ring[c] == 4) {
      if (bx == 128) return (const void*)&kb_lb2d<St, R, 128, 4, 2, FORM>;
      if (bx == 192) return (const void*)&kb_lb2d<St, R, 192, 4, 2, FORM>;
      if (bx == 256) return (const void*)&kb_lb2d<St, R, 256, 4, 2, FORM>;
      return (const void*)&kb_lb2d<St, R, 64, 4, 2, FORM>;
    }
    if (bx == 128) return (const void*)&kb_lb2d<St, R, 128, 3, WPE3, FORM>;
    if (bx == 192) return (const void*)&kb_lb2d<St, R, 192, 3, WPE3, FORM>;
    if (bx == 256) return (const void*)&kb_lb2d<St, R, 256, 3, WPE3, FORM>;
    return (const void*)&kb_lb2d<St, R, 64, 3, WPE3, FORM>;
  }
  // the divergence form's extra LDS ring leaves room for two waves per SIMD
  const void* lb_kernel(int c) const { return force_form ? lb_kernel_f<2, 1>(c) : lb_kernel_f<3, 0>(c); }
  int resident(const void* k, int threads) const {
    int per_cu = 0, ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0) != hipSuccess || per_cu <= 0 ||
        ncu <= 0)
      return 1024;
    return per_cu * ncu;
  }

  // device tables and launch plan; graph capture
  int prepare() {
    const int n = (int)mem.size();
    if (n == 0) return LBIB_EINVAL;
    for (auto m : mem)
      if (!m->ready || m->cur != mem[0]->cur) return LBIB_ESTATE;
    std::vector<BMember<St>> T(n);
    std::vector<int2> mems;
    std::vector<int> mpre(n + 1, 0), cm(NCLS * n, 0), bpre(NCLS * (n + 1), 0);
    std::vector<int> cls(n);
    long long rows[NCLS] = {0, 0, 0};
    for (int i = 0; i < n; i++) {
      cls[i] = size_class(mem[i]->p.nx);
      const int W = cls_bx[cls[i]] - 4;
      rows[cls[i]] += (long long)((mem[i]->p.nx + W - 1) / W) * mem[i]->p.ny;
    }
    for (int c = 0; c < NCLS; c++) {
      const int slots = resident(lb_kernel(c), cls_bx[c]);
      lseg[c] = cls_seg[c] > 0 ? cls_seg[c] : (int)std::max<long long>(4, (rows[c] + slots - 1) / slots);
      ncm[c] = 0;
    }
    long long tiles = 0;
    for (int i = 0; i < n; i++) {
      Mem* m = mem[i];
      const int c = cls[i];
      BMember<St>& B = T[i];
      B.P = m->P;
      const int W = cls_bx[c] - 4;
      B.P.seg = std::min(lseg[c], m->p.ny);
      B.P.nstrip = (m->p.nx + W - 1) / W;
      B.P.nseg = (m->p.ny + B.P.seg - 1) / B.P.seg;
      B.P.nxcd = 1;
      B.a = m->store(0);
      B.b = m->store(1);
      B.md = m->memdev();
      B.tm = m->tilemap();
      B.ca = m->coup_args(1);
      B.Ifield = m->template at<double>(m->L.Ifield);
      B.fib = m->template at<long long>(m->L.fib);
      B.force = m->template at<double>(m->L.force);
      for (int k = 0; k < m->K; k++) mems.push_back(make_int2(i, k));
      mpre[i + 1] = mpre[i] + m->M;
      tiles += m->L.ntiles * (m->K > 0);
      const int q = ncm[c]++;
      cm[c * n + q] = i;
      bpre[c * (n + 1) + q + 1] = bpre[c * (n + 1) + q] + B.P.nstrip * B.P.nseg;
    }
    nmems = (int)mems.size();
    Mtot = mpre[n];
    cgrid = (int)std::max<long long>(1, std::min<long long>(tiles, 4096));
    for (int c = 0; c < NCLS; c++) {
      const int items = bpre[c * (n + 1) + ncm[c]];
      lgrid[c] = std::max(1, items);  // one item per workgroup
    }
    hipStream_t st = stream;
    HIPCHK(hipMemcpyAsync(ws + off_tab, T.data(), T.size() * sizeof(BMember<St>), hipMemcpyHostToDevice, st));
    if (!mems.empty())
      HIPCHK(hipMemcpyAsync(ws + off_mems, mems.data(), mems.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws + off_mpre, mpre.data(), mpre.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws + off_cm, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ws + off_bpre, bpre.data(), bpre.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    drop_graphs();
    if (use_graph) {
      graph_ok = true;
      for (int par = 0; par < 2 && graph_ok; par++) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) {
          graph_ok = false;
          break;
        }
        launch_all(par);
        if (hipStreamEndCapture(st, &g) != hipSuccess || !g ||
            hipGraphInstantiate(&gexec[par], g, nullptr, nullptr, 0) != hipSuccess)
          graph_ok = false;
        if (g) (void)hipGraphDestroy(g);
      }
      if (!graph_ok) {
        drop_graphs();
        (void)hipGetLastError();  // a stream that cannot be captured: launch directly
      }
    }
    dirty = false;
    return LBIB_OK;
  }

  void launch_all(int parity) {
    const int n = (int)mem.size();
    BMember<St>* T = at<BMember<St>>(off_tab);
    const int* mpre = at<int>(off_mpre);
    hipLaunchKernelGGL(kb_begin<St>, dim3((n + 63) / 64), dim3(64), 0, stream, T, n);
    if (nmems > 0) {
      hipLaunchKernelGGL((kb_tiles<St, 256>), dim3(nmems), dim3(256), 0, stream, (const BMember<St>*)T,
                         (const int2*)at<int2>(off_mems));
      hipLaunchKernelGGL((kb_coupling2d<St, R, COUP_THREADS>), dim3(cgrid), dim3(COUP_THREADS), 0, stream,
                         (const BMember<St>*)T, n, parity);
      hipLaunchKernelGGL(kb_forcespread2d<St>, dim3((16 * Mtot + 255) / 256), dim3(256), 0, stream,
                         (const BMember<St>*)T, mpre, n);
    }
    for (int c = 0; c < NCLS; c++) {
      if (!ncm[c]) continue;
      const int* cmc = at<int>(off_cm) + c * n;
      const int* bp = at<int>(off_bpre) + c * (n + 1);
      const BMember<St>* Tc = T;
#define KB_LAUNCH(BXV, NSV, WPEV)                                                                    \
  do {                                                                                               \
    if (force_form == 1)                                                                             \
      hipLaunchKernelGGL((kb_lb2d<St, R, BXV, NSV, 2, 1>), dim3(lgrid[c]), dim3(BXV), 0, stream, Tc, cmc, bp, \
                         ncm[c], parity);                                                            \
    else                                                                                             \
      hipLaunchKernelGGL((kb_lb2d<St, R, BXV, NSV, WPEV>), dim3(lgrid[c]), dim3(BXV), 0, stream, Tc, cmc, bp, \
                         ncm[c], parity);                                                            \
  } while (0)
      if (cls_ring[c] == 4) {
        if (cls_bx[c] == 128) KB_LAUNCH(128, 4, 2);
        else if (cls_bx[c] == 192) KB_LAUNCH(192, 4, 2);
        else if (cls_bx[c] == 256) KB_LAUNCH(256, 4, 2);
        else KB_LAUNCH(64, 4, 2);
      } else {
        if (cls_bx[c] == 128) KB_LAUNCH(128, 3, 3);
        else if (cls_bx[c] == 192) KB_LAUNCH(192, 3, 3);
        else if (cls_bx[c] == 256) KB_LAUNCH(256, 3, 3);
        else KB_LAUNCH(64, 3, 3);
      }
#undef KB_LAUNCH
    }
    if (nmems > 0)
      hipLaunchKernelGGL((kb_interp2d<St, R>), dim3((16 * Mtot + 255) / 256), dim3(256), 0, stream,
                         (const BMember<St>*)T, mpre, n, parity);
  }

  int step() override {
    if (dirty) {
      int rc = prepare();
      if (rc) return rc;
    }
    const int parity = mem[0]->cur;
    if (graph_ok) {
      if (hipGraphLaunch(gexec[parity], stream) != hipSuccess) return LBIB_EHIP;
    } else {
      launch_all(parity);
    }
    for (auto m : mem) {
      m->cur = 1 - m->cur;
      m->steps++;
    }
    return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
  }
};

lbib_sim* make_engine(const lbib_params* p) {
  if (p->lattice == LBIB_D2Q9) {
    switch (p->storage) {
      case LBIB_FP32: return new (std::nothrow) Engine2D<MixStore<9>, float>();
      case LBIB_FP64: return new (std::nothrow) Engine2D<PlainStore<double, 9>, double>();
      case LBIB_FP16: return new (std::nothrow) Engine2D<Split16Store<__half, 9>, float>();
      case LBIB_BF16: return new (std::nothrow) Engine2D<Split16Store<__hip_bfloat16, 9>, float>();
    }
  } else {
    switch (p->storage) {
      case LBIB_FP32: return new (std::nothrow) Engine3D<MixStore<19>, float>();
      case LBIB_FP64: return new (std::nothrow) Engine3D<PlainStore<double, 19>, double>();
      case LBIB_FP16: return new (std::nothrow) Engine3D<Split16Store<__half, 19>, float>();
      case LBIB_BF16: return new (std::nothrow) Engine3D<Split16Store<__hip_bfloat16, 19>, float>();
    }
  }
  return nullptr;
}

}  // namespace

// ---------------------------------------------------------------------------
namespace {

// closed-mesh topology on the host: edges with their two triangles, the
// triangle across each edge, and the vertex -> triangle lists.  Returns
// LBIB_EINVAL for an index out of range, a degenerate triangle, or an edge
// that does not have exactly two triangles (open or non-manifold mesh).
struct MeshTopo {
  std::vector<int> edge;   // 4 per edge: a < b, t1, t2 (local ids)
  std::vector<int> tadj;   // 3 per triangle
  std::vector<int> vtoff;  // n + 1
  std::vector<int> vt;
};

int mesh_topology(int n, int nt, const int* tri, MeshTopo& mt) {
  std::vector<std::pair<long long, int>> keys;  // (edge key, 3 t + k)
  keys.reserve((size_t)3 * nt);
  for (int t = 0; t < nt; t++) {
    const int* v = tri + 3 * t;
    for (int k = 0; k < 3; k++) {
      if (v[k] < 0 || v[k] >= n) return LBIB_EINVAL;
    }
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) return LBIB_EINVAL;
    for (int k = 0; k < 3; k++) {
      const int a = v[k], b = v[(k + 1) % 3];
      keys.push_back({(long long)std::min(a, b) * n + std::max(a, b), 3 * t + k});
    }
  }
  std::sort(keys.begin(), keys.end());
  mt.tadj.assign((size_t)3 * nt, -1);
  mt.edge.clear();
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j].first == keys[i].first) j++;
    if (j - i != 2) return LBIB_EINVAL;
    const int s0 = keys[i].second, s1 = keys[i + 1].second;
    const int t1 = s0 / 3, t2 = s1 / 3;
    mt.tadj[s0] = t2;
    mt.tadj[s1] = t1;
    mt.edge.push_back((int)(keys[i].first / n));
    mt.edge.push_back((int)(keys[i].first % n));
    mt.edge.push_back(t1);
    mt.edge.push_back(t2);
    i = j;
  }
  mt.vtoff.assign((size_t)n + 1, 0);
  for (int q = 0; q < 3 * nt; q++) mt.vtoff[tri[q] + 1]++;
  for (int v = 0; v < n; v++) mt.vtoff[v + 1] += mt.vtoff[v];
  mt.vt.assign((size_t)3 * nt, 0);
  std::vector<int> fill(mt.vtoff.begin(), mt.vtoff.end() - 1);
  for (int t = 0; t < nt; t++)
    for (int k = 0; k < 3; k++) mt.vt[fill[tri[3 * t + k]]++] = t;
  return LBIB_OK;
}

}  // namespace

namespace {

// common set-up of a simulation object on its workspace
int init_sim(lbib_sim* s, const lbib_params* p, const Layout& L, char* ws, hipStream_t stream) {
  s->p = *p;
  s->L = L;
  s->ws = (char*)ws;
  s->stream = (hipStream_t)stream;
  s->Q = p->lattice == LBIB_D2Q9 ? 9 : 19;
  s->D = p->lattice == LBIB_D2Q9 ? 2 : 3;
  s->N = (long long)p->nx * p->ny * p->nz;
  s->r_cut = p->r_cut > 0 ? p->r_cut : 17.0 * p->alpha;
  s->seg = 0;  // automatic: one resident round of workgroups
  // D2Q9 starts in the divergence form of the thermodynamic force, which
  // conserves the lattice momentum exactly (D3Q19 has the potential form only)
  s->force_form = s->D == 2 ? 1 : 0;
  s->setup();
  // zero the maps, accumulators and counters (fill kernels would do as well;
  // memset is only used here, outside any step)
  hipStream_t st = s->stream;
  if (hipMemsetAsync(s->ws + L.fib, 0, (size_t)s->N * s->D * 8, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.tflag, 0, (size_t)L.ntiles * 4, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.tstate, 0, 64, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.Facc, 0, (size_t)std::max(p->max_markers, 1) * 3 * 8, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.status, 0, 64, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.force, 0, (size_t)s->N * s->D * 8, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.moff, 0, 4, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.Ifield, 0, (size_t)s->N * 8, st) != hipSuccess ||
      hipMemsetAsync(s->ws + L.mbox, 0, (size_t)std::max(p->max_membranes, 1) * 64, st) != hipSuccess)
    return LBIB_EHIP;
  if (hipMemsetAsync(s->ws + L.ckey, 0xff, (size_t)(s->D == 2 ? COUP_CACHE : COUP3_CACHE) * s->N * 4, st) !=
      hipSuccess)
    return LBIB_EHIP;
  // the tile flags start at 0 and the stamp at 1: no tile is active until a
  // membrane's tile pass flags it (a simulation without membranes never
  // reads the profile or force maps)
  static const int stamp0[3] = {0, 1, 0};
  if (hipMemcpyAsync(s->ws + L.tstate, stamp0, sizeof(stamp0), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return LBIB_EHIP;
  return LBIB_OK;
}

}  // namespace

// C ABI
extern "C" {

int lbib_workspace_bytes(const lbib_params* p, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return LBIB_EINVAL;
  *bytes = make_layout(p).total;
  return LBIB_OK;
}

int lbib_create(const lbib_params* p, void* ws, size_t ws_bytes, void* stream, lbib_sim** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!ws || !out || ((uintptr_t)ws % kAlign) != 0) return LBIB_EINVAL;
  Layout L = make_layout(p);
  if (ws_bytes < L.total) return LBIB_ENOMEM;
  lbib_sim* s = make_engine(p);
  if (!s) return LBIB_ENOMEM;
  rc = init_sim(s, p, L, (char*)ws, (hipStream_t)stream);
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return LBIB_OK;
}


int lbib_add_membrane(lbib_sim* s, int n, const double* X, int n_elems, const int* conn, double ks,
                      double kb, int* id) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !X || n < 3) return LBIB_EINVAL;
  if (s->ready) return LBIB_ESTATE;
  if (s->D == 2 && (n_elems != 0 || conn)) return LBIB_EINVAL;
  if (s->D == 3 && (n_elems < 4 || !conn)) return LBIB_EINVAL;
  if (!(ks >= 0) || !(kb >= 0)) return LBIB_EINVAL;
  if (s->K + 1 > s->p.max_membranes || s->M + n > s->p.max_markers) return LBIB_ENOMEM;
  if (s->D == 3 && s->ntri + n_elems > s->p.max_elems) return LBIB_ENOMEM;
  for (int i = 0; i < n * s->D; i++)
    if (!std::isfinite(X[i])) return LBIB_EINVAL;
  std::vector<double> X3((size_t)3 * n, 0.0), rest(n, 1.0);
  for (int l = 0; l < n; l++)
    for (int a = 0; a < s->D; a++) X3[3 * l + a] = X[(size_t)l * s->D + a];
  if (s->D == 2) {
    for (int l = 0; l < n; l++) {
      const int m = (l + 1) % n;
      rest[l] = std::hypot(X3[3 * m] - X3[3 * l], X3[3 * m + 1] - X3[3 * l + 1]);
      if (!(rest[l] > 0)) return LBIB_EINVAL;
    }
  }
  const int off = s->M;
  hipStream_t st = s->stream;
  MeshTopo mt;
  std::vector<int> tri_g, edge_g, tadj_g, tedge_g, vtoff_g, vt_g, emem;
  std::vector<double> erest;
  if (s->D == 3) {
    int rc = mesh_topology(n, n_elems, conn, mt);
    if (rc) return rc;
    const int ne = (int)mt.edge.size() / 4;
    if (s->nedge + ne > s->L.maxE) return LBIB_ENOMEM;
    // global ids: markers offset by M, triangles by T
    tri_g.resize((size_t)3 * n_elems);
    for (int q = 0; q < 3 * n_elems; q++) tri_g[q] = conn[q] + off;
    tadj_g.resize(mt.tadj.size());
    for (size_t q = 0; q < mt.tadj.size(); q++) tadj_g[q] = mt.tadj[q] + s->ntri;
    edge_g.resize(mt.edge.size());
    erest.resize(ne);
    for (int e = 0; e < ne; e++) {
      const int a = mt.edge[4 * e], b = mt.edge[4 * e + 1];
      edge_g[4 * e] = a + off;
      edge_g[4 * e + 1] = b + off;
      edge_g[4 * e + 2] = mt.edge[4 * e + 2] + s->ntri;
      edge_g[4 * e + 3] = mt.edge[4 * e + 3] + s->ntri;
      erest[e] = std::sqrt((X3[3 * b] - X3[3 * a]) * (X3[3 * b] - X3[3 * a]) +
                           (X3[3 * b + 1] - X3[3 * a + 1]) * (X3[3 * b + 1] - X3[3 * a + 1]) +
                           (X3[3 * b + 2] - X3[3 * a + 2]) * (X3[3 * b + 2] - X3[3 * a + 2]));
      if (!(erest[e] > 0)) return LBIB_EINVAL;
    }
    // each triangle's edges, by the vertex opposite them (the triangle laws)
    tedge_g.assign((size_t)3 * n_elems, -1);
    for (int e = 0; e < ne; e++)
      for (int side = 2; side < 4; side++) {
        const int t = mt.edge[4 * e + side];
        for (int k = 0; k < 3; k++) {
          const int v = conn[3 * t + k];
          if (v != mt.edge[4 * e] && v != mt.edge[4 * e + 1]) tedge_g[3 * t + k] = s->nedge + e;
        }
      }
    for (int q = 0; q < 3 * n_elems; q++)
      if (tedge_g[q] < 0) return LBIB_EINVAL;
    emem.assign(ne, s->K);
    const int vbase = s->vtoff.back();
    vtoff_g.resize(n);
    for (int v = 0; v < n; v++) vtoff_g[v] = mt.vtoff[v + 1] + vbase;  // entries off + 1 .. off + n
    vt_g.resize(mt.vt.size());
    for (size_t q = 0; q < mt.vt.size(); q++) vt_g[q] = mt.vt[q] + s->ntri;
  }
  std::vector<int> mid(n, s->K);
  HIPCHK(hipMemcpyAsync(s->ws + s->L.X + (size_t)off * 24, X3.data(), (size_t)n * 24, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(s->ws + s->L.U + (size_t)off * 24, 0, (size_t)n * 24, st));
  HIPCHK(hipMemsetAsync(s->ws + s->L.F + (size_t)off * 24, 0, (size_t)n * 24, st));
  HIPCHK(hipMemcpyAsync(s->ws + s->L.rest + (size_t)off * 8, rest.data(), (size_t)n * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->ws + s->L.mid + (size_t)off * 4, mid.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->ws + s->L.ks + (size_t)s->K * 8, &ks, 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->ws + s->L.kb + (size_t)s->K * 8, &kb, 8, hipMemcpyHostToDevice, st));
  const int law0 = 0;
  HIPCHK(hipMemcpyAsync(s->ws + s->L.law + (size_t)s->K * 4, &law0, 4, hipMemcpyHostToDevice, st));
  s->moff.push_back(off + n);
  HIPCHK(hipMemcpyAsync(s->ws + s->L.moff, s->moff.data(), s->moff.size() * 4, hipMemcpyHostToDevice, st));
  if (s->D == 3) {
    const int ne = (int)erest.size();
    char* w = s->ws;
    HIPCHK(hipMemcpyAsync(w + s->L.tri + (size_t)s->ntri * 12, tri_g.data(), tri_g.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.tadj + (size_t)s->ntri * 12, tadj_g.data(), tadj_g.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.tedge + (size_t)s->ntri * 12, tedge_g.data(), tedge_g.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.edge + (size_t)s->nedge * 16, edge_g.data(), edge_g.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.erest + (size_t)s->nedge * 8, erest.data(), erest.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.emem + (size_t)s->nedge * 4, emem.data(), emem.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.vt + (size_t)s->vtoff.back() * 4, vt_g.data(), vt_g.size() * 4, hipMemcpyHostToDevice, st));
    s->toff.push_back(s->ntri + n_elems);
    s->coff.push_back(s->coff.back() + (n_elems + CL3 - 1) / CL3);
    s->eoff.push_back(s->nedge + ne);
    for (int v = 0; v < n; v++) s->vtoff.push_back(vtoff_g[v]);
    HIPCHK(hipMemcpyAsync(w + s->L.toff, s->toff.data(), s->toff.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.eoff, s->eoff.data(), s->eoff.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.coff, s->coff.data(), s->coff.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(w + s->L.vtoff, s->vtoff.data(), s->vtoff.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // host vectors go out of scope
    s->ntri += n_elems;
    s->nedge += ne;
  }
  HIPCHK(hipStreamSynchronize(st));
  if (id) *id = s->K;
  s->K += 1;
  s->M += n;
  if (s->owner) s->owner->mark_dirty();
  return LBIB_OK;
}

int lbib_set_rest(lbib_sim* s, int id, const double* rest) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !rest || id < 0 || id >= s->K) return LBIB_EINVAL;
  hipStream_t st = s->stream;
  if (s->D == 2) {
    const int b = s->moff[id], n = s->moff[id + 1] - b;
    for (int l = 0; l < n; l++)
      if (!(rest[l] > 0) || !std::isfinite(rest[l])) return LBIB_EINVAL;
    HIPCHK(hipMemcpyAsync(s->ws + s->L.rest + (size_t)b * 8, rest, (size_t)n * 8, hipMemcpyHostToDevice, st));
  } else {
    const int b = s->eoff[id], n = s->eoff[id + 1] - b;
    for (int e = 0; e < n; e++)
      if (!(rest[e] > 0) || !std::isfinite(rest[e])) return LBIB_EINVAL;
    HIPCHK(hipMemcpyAsync(s->ws + s->L.erest + (size_t)b * 8, rest, (size_t)n * 8, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return LBIB_OK;
}

int lbib_set_fields(lbib_sim* s, const double* rho, const double* phi, const double* psi,
                    const double* ux, const double* uy, const double* uz) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !rho || !phi || !psi) return LBIB_EINVAL;
  const long long N = s->N;
  for (long long n = 0; n < N; n++)
    if (!(rho[n] > 0) || !std::isfinite(phi[n]) || !std::isfinite(psi[n])) return LBIB_EINVAL;
  double* stage = s->at<double>(s->L.stage);
  hipStream_t st = s->stream;
  HIPCHK(hipMemcpyAsync(stage, rho, N * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(stage + N, phi, N * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(stage + 2 * N, psi, N * 8, hipMemcpyHostToDevice, st));
  if (ux)
    HIPCHK(hipMemcpyAsync(stage + 3 * N, ux, N * 8, hipMemcpyHostToDevice, st));
  else
    HIPCHK(hipMemsetAsync(stage + 3 * N, 0, N * 8, st));
  if (uy)
    HIPCHK(hipMemcpyAsync(stage + 4 * N, uy, N * 8, hipMemcpyHostToDevice, st));
  else
    HIPCHK(hipMemsetAsync(stage + 4 * N, 0, N * 8, st));
  if (s->D == 3) {
    if (uz)
      HIPCHK(hipMemcpyAsync(stage + 5 * N, uz, N * 8, hipMemcpyHostToDevice, st));
    else
      HIPCHK(hipMemsetAsync(stage + 5 * N, 0, N * 8, st));
  }
  s->cur = 0;
  int rc = s->init(stage);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  s->ready = true;
  s->steps = 0;
  if (s->owner) s->owner->mark_dirty();
  return LBIB_OK;
}

int lbib_step(lbib_sim* s, int n) {
  if (!s || n < 0) return LBIB_EINVAL;
  if (!s->ready || s->owner) return LBIB_ESTATE;  // batch members step with their batch
  for (int k = 0; k < n; k++) {
    int rc = s->step();
    if (rc) return rc;
    s->steps++;
  }
  return LBIB_OK;
}

long long lbib_steps_done(const lbib_sim* s) { return s ? s->steps : -1; }

int lbib_set_launch(lbib_sim* s, int block_x, int seg, int nxcd, int ring) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s) return LBIB_EINVAL;
  if (ring != 0 && ring != 3 && ring != 4) return LBIB_EINVAL;
  if (s->D == 3) {
    if (block_x != 0 && block_x != 16 && block_x != 32 && block_x != 64) return LBIB_EINVAL;
  } else if (block_x != 0 && block_x != 64 && block_x != 128 && block_x != 192 && block_x != 256) {
    return LBIB_EINVAL;
  }
  if (seg < -1 || nxcd < -1 || nxcd > 64) return LBIB_EINVAL;
  if (ring) s->ring = ring;
  if (block_x) (s->D == 3 ? s->tx3 : s->bx) = block_x;
  if (seg > 0) s->seg = std::max(1, std::min(seg, s->D == 3 ? s->p.nz : s->p.ny));
  if (seg < 0) s->seg = 0;  // back to automatic
  if (nxcd > 0) s->nxcd = nxcd;
  if (nxcd < 0) s->nxcd = 0;  // back to automatic
  return LBIB_OK;
}

int lbib_set_overlap(lbib_sim* s, int on) {
  if (!s || s->is_batch() || on < -1 || on > 1) return LBIB_EINVAL;
  s->overlap = on > 0 ? 1 : 0;
  return LBIB_OK;
}

int lbib_set_membrane_law(lbib_sim* s, int id, int law) {
  if (!s || s->is_batch() || id < 0 || id >= s->K || law < 0 || law > 2) return LBIB_EINVAL;
  HIPCHK(hipMemcpyAsync(s->ws + s->L.law + (size_t)id * 4, &law, 4, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (law != 0) s->any_law = true;
  return LBIB_OK;
}

int lbib_set_external_force(lbib_sim* s, double fx, double fy, double fz) {
  if (!s || s->is_batch() || !std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(fz) ||
      (s->D == 2 && fz != 0.0))
    return LBIB_EINVAL;
  s->fext[0] = fx;
  s->fext[1] = fy;
  s->fext[2] = fz;
  s->setup();
  if (s->owner) s->owner->mark_dirty();  // the batch copies the member's parameters
  return LBIB_OK;
}

int lbib_set_densities(lbib_sim* s, double m1, double m2, double m3) {
  if (!s || s->is_batch()) return LBIB_EINVAL;
  const double m[3] = {m1, m2, m3};
  for (int k = 0; k < 3; k++)
    if (!std::isfinite(m[k]) || !(m[k] > 0.0)) return LBIB_EINVAL;
  if (s->ready) return LBIB_ESTATE;  // the populations hold the old map's pressure
  for (int k = 0; k < 3; k++) s->mw[k] = m[k];
  s->setup();
  if (s->owner) s->owner->mark_dirty();  // the batch copies the member's parameters
  return LBIB_OK;
}

int lbib_set_coupling_cache(lbib_sim* s, int on) {
  if (!s || on < 0 || on > 1) return LBIB_EINVAL;
  if (s->is_batch()) {
    for (int k = 0;; k++) {
      lbib_sim* m = nullptr;
      if (lbib_batch_member(s, k, &m) != LBIB_OK) break;
      m->coup_cache = on;
    }
    s->coup_cache = on;
    s->mark_dirty();
    return LBIB_OK;
  }
  if (on && !s->coup_cache && s->drop_coupling_cache() != LBIB_OK) return LBIB_EHIP;  // stale entries
  s->coup_cache = on;
  if (s->owner) s->owner->mark_dirty();
  return LBIB_OK;
}

int lbib_set_force_form(lbib_sim* s, int form) {
  if (!s || s->owner || s->D != 2 || form < 0 || form > 1) return LBIB_EINVAL;
  if (s->force_form != form && s->is_batch()) s->mark_dirty();  // new launch plan and graphs
  s->force_form = form;
  return LBIB_OK;
}

int lbib_get_launch(const lbib_sim* s, int* block_x, int* seg, int* nxcd, int* ring) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s) return LBIB_EINVAL;
  if (ring) *ring = s->ring;
  if (block_x) *block_x = s->D == 3 ? s->tx3 : s->bx;
  if (seg) *seg = s->seg;
  if (nxcd) *nxcd = s->nxcd;
  return LBIB_OK;
}

int lbib_timing_enable(lbib_sim* s, int on) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s) return LBIB_EINVAL;
  int rc = s->timing_flush();
  if (rc) return rc;
  s->timing = on & 15;
  s->timed_steps = 0;
  for (double& v : s->timed_ms) v = 0;
  return LBIB_OK;
}

int lbib_timing_read(lbib_sim* s, double* ms, int n, int* steps) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || n < 0 || n > 4 || (n > 0 && !ms)) return LBIB_EINVAL;
  int rc = s->timing_flush();
  if (rc) return rc;
  for (int k = 0; k < n; k++) ms[k] = s->timed_ms[k];
  if (steps) *steps = s->timed_steps;
  return LBIB_OK;
}

int lbib_get_fields(lbib_sim* s, double* rho, double* c1, double* c2, double* c3, double* ux,
                    double* uy, double* uz) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s) return LBIB_EINVAL;
  if (!s->ready) return LBIB_ESTATE;
  double* stage = s->at<double>(s->L.stage);
  int rc = s->moments(stage);
  if (rc) return rc;
  const long long N = s->N;
  double* outs[7] = {rho, c1, c2, c3, ux, uy, s->D == 3 ? uz : nullptr};
  for (int k = 0; k < 7; k++)
    if (outs[k]) HIPCHK(hipMemcpyAsync(outs[k], stage + k * N, N * 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return LBIB_OK;
}

int lbib_get_membrane(lbib_sim* s, int id, double* X, double* U, double* F) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || id < 0 || id >= s->K) return LBIB_EINVAL;
  const int b = s->moff[id], n = s->moff[id + 1] - b;
  std::vector<double> buf((size_t)3 * n);
  const size_t offs[3] = {s->L.X, s->L.U, s->L.F};
  double* outs[3] = {X, U, F};
  for (int k = 0; k < 3; k++) {
    if (!outs[k]) continue;
    HIPCHK(hipMemcpyAsync(buf.data(), s->ws + offs[k] + (size_t)b * 24, (size_t)n * 24, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int l = 0; l < n; l++)
      for (int a = 0; a < s->D; a++) outs[k][(size_t)l * s->D + a] = buf[3 * l + a];
  }
  return LBIB_OK;
}

int lbib_energy(lbib_sim* s, lbib_energies* out) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !out) return LBIB_EINVAL;
  if (!s->ready) return LBIB_ESTATE;
  double* stage = s->at<double>(s->L.stage);
  double* part = s->at<double>(s->L.part);
  int rc = s->coupling(0);  // profile I at the current markers
  if (rc) return rc;
  rc = s->moments(stage);
  if (rc) return rc;
  long long nblk = 0;
  rc = s->energy_nodes(part, &nblk);
  if (rc) return rc;
  double* sums = s->at<double>(s->L.memE);
  hipLaunchKernelGGL(k_sum_rows<256>, dim3(1), dim3(256), 0, s->stream, (const double*)part, nblk, 8, sums);
  double host[8];
  HIPCHK(hipMemcpyAsync(host, sums, 64, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  for (int k = 0; k < 3; k++) out->mass[k] = host[k];
  out->F_bulk = host[3];
  out->F_grad = host[4];
  out->E_c = host[5];
  out->E_kin = host[6];
  out->p_ideal = host[7];
  out->E_s = out->E_b = 0.0;
  if (s->K > 0) {
    double* me = part + ((s->N + 255) / 256 + 1) * 8;
    long long rows = 0;
    rc = s->mem_energy(me, &rows);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_rows<256>, dim3(1), dim3(256), 0, s->stream, (const double*)me, rows, 2,
                       sums);
    double h2[2];
    HIPCHK(hipMemcpyAsync(h2, sums, 16, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    out->E_s = h2[0];
    out->E_b = h2[1];
  }
  return LBIB_OK;
}

int lbib_check(lbib_sim* s) {
  if (!s) return LBIB_EINVAL;
  if (s->is_batch()) {
    for (auto m : static_cast<BatchEngine2D*>(s)->mem) {
      int rc = lbib_check(m);
      if (rc) return rc;
    }
    return LBIB_OK;
  }
  if (!s->ready) return LBIB_ESTATE;
  int* st = s->at<int>(s->L.status);
  HIPCHK(hipMemsetAsync(st + 8, 0, 4, s->stream));
  int rc = s->check(st + 8);
  if (rc) return rc;
  int host[9];
  HIPCHK(hipMemcpyAsync(host, st, 36, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (host[8]) return LBIB_ENONFINITE;
  if (host[0] || host[1]) return LBIB_EUNSTABLE;
  return LBIB_OK;
}

int lbib_device_view(lbib_sim* s, int field, void** ptr, size_t* elems) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !ptr || !elems) return LBIB_EINVAL;
  switch (field) {
    case 0:
      *ptr = s->ws + s->L.pops[s->cur];
      *elems = s->L.pop_bytes;
      return LBIB_OK;
    case 1:
      *ptr = s->ws + s->L.Ifield;
      *elems = (size_t)s->N;
      return LBIB_OK;
    case 2:
      *ptr = s->ws + s->L.X;
      *elems = (size_t)s->M * 3;
      return LBIB_OK;
  }
  return LBIB_EINVAL;
}

// checkpoint header: a tag and the parameters a checkpoint must match
namespace {
constexpr long long CKPT_TAG = 0x31504b4342494c42LL;  // "BLIBCKP1" read as little-endian bytes
constexpr int CKPT_WORDS = 12;
void ckpt_header(const lbib_sim* s, long long* h) {
  const int form = s->owner ? s->owner->force_form : s->force_form;
  // last word: the component densities' bit patterns mixed (0 when all are 1)
  unsigned long long dh = 0;
  if (s->mw[0] != 1.0 || s->mw[1] != 1.0 || s->mw[2] != 1.0)
    for (int k = 0; k < 3; k++) {
      unsigned long long bits;
      memcpy(&bits, &s->mw[k], 8);
      dh = (dh ^ bits) * 0x100000001b3ULL + 0x9e3779b97f4a7c15ULL;
    }
  const long long v[CKPT_WORDS] = {CKPT_TAG, s->steps, (long long)s->M, (long long)s->K, s->p.nx, s->p.ny,
                                   s->p.nz, (long long)s->Q, (long long)s->p.storage, (long long)form,
                                   (long long)s->L.pop_bytes, (long long)dh};
  for (int k = 0; k < CKPT_WORDS; k++) h[k] = v[k];
}
}  // namespace

int lbib_save(lbib_sim* s, void* buf, size_t* bytes) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !bytes) return LBIB_EINVAL;
  if (!s->ready) return LBIB_ESTATE;
  const size_t H = CKPT_WORDS * 8;
  const size_t need = H + s->L.pop_bytes + (size_t)s->M * 24 * 3;
  if (!buf) {
    *bytes = need;
    return LBIB_OK;
  }
  if (*bytes < need) return LBIB_ENOMEM;
  char* o = (char*)buf;
  long long hdr[CKPT_WORDS];
  ckpt_header(s, hdr);
  memcpy(o, hdr, H);
  HIPCHK(hipMemcpyAsync(o + H, s->ws + s->L.pops[s->cur], s->L.pop_bytes, hipMemcpyDeviceToHost, s->stream));
  const size_t offs[3] = {s->L.X, s->L.U, s->L.F};
  for (int k = 0; k < 3; k++)
    HIPCHK(hipMemcpyAsync(o + H + s->L.pop_bytes + (size_t)k * s->M * 24, s->ws + offs[k],
                          (size_t)s->M * 24, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  *bytes = need;
  return LBIB_OK;
}

int lbib_load(lbib_sim* s, const void* buf, size_t bytes) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s || !buf) return LBIB_EINVAL;
  const size_t H = CKPT_WORDS * 8;
  const size_t need = H + s->L.pop_bytes + (size_t)s->M * 24 * 3;
  if (bytes < need) return LBIB_EINVAL;
  const char* o = (const char*)buf;
  long long hdr[CKPT_WORDS], want[CKPT_WORDS];
  memcpy(hdr, o, H);
  ckpt_header(s, want);
  // every word but the step count must match: tag, markers, membranes,
  // lattice size, Q, storage, force form, population bytes and densities
  for (int k = 0; k < CKPT_WORDS; k++)
    if (k != 1 && hdr[k] != want[k]) return LBIB_EINVAL;
  if (hdr[1] < 0) return LBIB_EINVAL;
  HIPCHK(hipMemcpyAsync(s->ws + s->L.pops[s->cur], o + H, s->L.pop_bytes, hipMemcpyHostToDevice, s->stream));
  const size_t offs[3] = {s->L.X, s->L.U, s->L.F};
  for (int k = 0; k < 3; k++)
    HIPCHK(hipMemcpyAsync(s->ws + offs[k], o + H + s->L.pop_bytes + (size_t)k * s->M * 24,
                          (size_t)s->M * 24, hipMemcpyHostToDevice, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  s->steps = hdr[1];
  s->ready = true;
  if (s->drop_coupling_cache() != LBIB_OK || hipStreamSynchronize(s->stream) != hipSuccess) return LBIB_EHIP;
  if (s->owner) s->owner->mark_dirty();
  return LBIB_OK;
}

int lbib_debug_poke(lbib_sim* s, int field, long long idx, double value) {
  if (s && s->is_batch()) return LBIB_EINVAL;  // per-member calls go to the members
  if (!s) return LBIB_EINVAL;
  if (field == 2) {
    if (idx < 0 || idx >= (long long)s->M * 3) return LBIB_EINVAL;
    HIPCHK(hipMemcpyAsync(s->ws + s->L.X + idx * 8, &value, 8, hipMemcpyHostToDevice, s->stream));
    if (s->drop_coupling_cache() != LBIB_OK) return LBIB_EHIP;
    HIPCHK(hipStreamSynchronize(s->stream));
    return LBIB_OK;
  }
  if (field == 0) {
    // entry idx of the current buffer: FP32 planes (FP32 / 16-bit rest planes)
    // or FP64 planes (FP64 storage), in the storage's plane order
    char* base = s->ws + s->L.pops[s->cur];
    if (s->p.storage == LBIB_FP64) {
      if (idx < 0 || idx >= 3LL * s->Q * s->N) return LBIB_EINVAL;
      HIPCHK(hipMemcpyAsync(base + idx * 8, &value, 8, hipMemcpyHostToDevice, s->stream));
    } else {
      size_t off = 0;
      long long lim = (3LL * s->Q - 2) * s->N;
      if (s->p.storage == LBIB_FP16 || s->p.storage == LBIB_BF16) {
        // the rest planes: f_0 - w_0 (FP32, idx < N), then g_0 and h_0 (FP64)
        off = align_up((size_t)(3LL * (s->Q - 1) * s->N * 2));
        lim = 3 * s->N;
        if (idx >= s->N && idx < lim) {
          HIPCHK(hipMemcpyAsync(base + off + align_up((size_t)(s->N * 4)) + (idx - s->N) * 8, &value, 8,
                                hipMemcpyHostToDevice, s->stream));
          HIPCHK(hipStreamSynchronize(s->stream));
          return LBIB_OK;
        }
      }
      if (idx < 0 || idx >= lim) return LBIB_EINVAL;
      float v = (float)value;
      HIPCHK(hipMemcpyAsync(base + off + idx * 4, &v, 4, hipMemcpyHostToDevice, s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return LBIB_OK;
  }
  return LBIB_EINVAL;
}

const char* lbib_strerror(int status) {
  switch (status) {
    case LBIB_OK: return "ok";
    case LBIB_EINVAL: return "invalid argument";
    case LBIB_ENOMEM: return "workspace or capacity too small";
    case LBIB_EHIP: return "HIP runtime error";
    case LBIB_ENONFINITE: return "non-finite population";
    case LBIB_EUNSTABLE: return "force out of range or membrane too large for the lattice";
    case LBIB_ESTATE: return "call out of order";
  }
  return "unknown status";
}

void lbib_destroy(lbib_sim* s) {
  if (s && !s->owner) delete s;  // batch members are destroyed with their batch
}

// ---------------------------------------------------------------------------
// batches of D2Q9 simulations

int lbib_batch_workspace_bytes(int n, const lbib_params* params, size_t* bytes) {
  if (n < 1 || n > BATCH_MAX || !params || !bytes) return LBIB_EINVAL;
  size_t tot = 0;
  int kmax = 0;
  for (int i = 0; i < n; i++) {
    int rc = validate(&params[i]);
    if (rc) return rc;
    if (params[i].lattice != LBIB_D2Q9 || params[i].storage != LBIB_FP32) return LBIB_EINVAL;
    tot += align_up(make_layout(&params[i]).total);
    kmax += params[i].max_membranes;
  }
  *bytes = BatchEngine2D::table_bytes(n, kmax) + tot;
  return LBIB_OK;
}

int lbib_batch_create(int n, const lbib_params* params, void* ws, size_t ws_bytes, void* stream,
                      lbib_sim** out) {
  size_t need = 0;
  int rc = lbib_batch_workspace_bytes(n, params, &need);
  if (rc) return rc;
  if (!ws || !out || ((uintptr_t)ws % kAlign) != 0) return LBIB_EINVAL;
  if (ws_bytes < need) return LBIB_ENOMEM;
  int kmax = 0;
  for (int i = 0; i < n; i++) kmax += params[i].max_membranes;
  BatchEngine2D* b = new (std::nothrow) BatchEngine2D();
  if (!b) return LBIB_ENOMEM;
  b->p = params[0];
  b->ws = (char*)ws;
  b->stream = (hipStream_t)stream;
  b->ready = true;
  b->off_tab = 0;
  b->off_mems = align_up((size_t)n * sizeof(BMember<BatchEngine2D::St>));
  b->off_mpre = b->off_mems + align_up((size_t)std::max(kmax, 1) * sizeof(int2));
  b->off_cm = b->off_mpre + align_up((size_t)(n + 1) * 4);
  b->off_bpre = b->off_cm + align_up((size_t)BatchEngine2D::NCLS * n * 4);
  size_t off = BatchEngine2D::table_bytes(n, kmax);
  for (int i = 0; i < n; i++) {
    Layout L = make_layout(&params[i]);
    BatchEngine2D::Mem* m = new (std::nothrow) BatchEngine2D::Mem();
    if (!m) {
      delete b;
      return LBIB_ENOMEM;
    }
    rc = init_sim(m, &params[i], L, (char*)ws + off, (hipStream_t)stream);
    m->owner = b;
    b->mem.push_back(m);
    if (rc) {
      delete b;
      return rc;
    }
    off += align_up(L.total);
  }
  *out = b;
  return LBIB_OK;
}

int lbib_batch_member(lbib_sim* batch, int k, lbib_sim** member) {
  if (!batch || !batch->is_batch() || !member) return LBIB_EINVAL;
  BatchEngine2D* b = static_cast<BatchEngine2D*>(batch);
  if (k < 0 || k >= (int)b->mem.size()) return LBIB_EINVAL;
  *member = b->mem[k];
  return LBIB_OK;
}

int lbib_batch_set_launch(lbib_sim* batch, int size_class, int block_x, int seg, int ring) {
  if (!batch || !batch->is_batch()) return LBIB_EINVAL;
  if (size_class < -1 || size_class >= BatchEngine2D::NCLS) return LBIB_EINVAL;
  if (block_x != 0 && block_x != 64 && block_x != 128 && block_x != 192 && block_x != 256) return LBIB_EINVAL;
  if (ring != 0 && ring != 3 && ring != 4) return LBIB_EINVAL;
  if (seg < -1) return LBIB_EINVAL;
  BatchEngine2D* b = static_cast<BatchEngine2D*>(batch);
  for (int c = 0; c < BatchEngine2D::NCLS; c++) {
    if (size_class >= 0 && c != size_class) continue;
    if (block_x) b->cls_bx[c] = block_x;
    if (ring) b->cls_ring[c] = ring;
    if (seg > 0) b->cls_seg[c] = seg;
    if (seg < 0) b->cls_seg[c] = 0;
  }
  b->dirty = true;
  return LBIB_OK;
}

int lbib_batch_get_launch(lbib_sim* batch, int size_class, int* block_x, int* seg, int* ring, int* members) {
  if (!batch || !batch->is_batch()) return LBIB_EINVAL;
  if (size_class < 0 || size_class >= BatchEngine2D::NCLS) return LBIB_EINVAL;
  BatchEngine2D* b = static_cast<BatchEngine2D*>(batch);
  if (block_x) *block_x = b->cls_bx[size_class];
  if (ring) *ring = b->cls_ring[size_class];
  if (seg) *seg = b->dirty ? b->cls_seg[size_class] : b->lseg[size_class];
  if (members) {
    int c = 0;
    for (auto m : b->mem) c += BatchEngine2D::size_class(m->p.nx) == size_class;
    *members = c;
  }
  return LBIB_OK;
}

int lbib_batch_graph(lbib_sim* batch, int on, int* active) {
  if (!batch || !batch->is_batch()) return LBIB_EINVAL;
  BatchEngine2D* b = static_cast<BatchEngine2D*>(batch);
  if (on >= 0) {
    b->use_graph = on != 0;
    b->dirty = true;
  }
  if (active) *active = (!b->dirty && b->graph_ok) ? 1 : 0;
  return LBIB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// warm-start network
struct lbib_mlp {
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int bmax = 0;
  long long t = 0;  // Adam steps taken
  size_t off_p, off_g, off_m, off_v, off_z1, off_a1, off_z2, off_a2, off_y, off_dy, off_d1, off_d2, off_part;
  template <typename T>
  T* at(size_t o) const { return reinterpret_cast<T*>(ws + o); }
};

namespace {

size_t mlp_layout(lbib_mlp* h, int B) {
  Carver c{nullptr};
  const size_t np = (size_t)MLP_NPARAM * 4;
  const size_t o_p = c.take(np), o_g = c.take(np), o_m = c.take(np), o_v = c.take(np);
  const size_t hid = (size_t)B * MLP_H * 4, out = (size_t)B * MLP_OUT * 4;
  const size_t o_z1 = c.take(hid), o_a1 = c.take(hid), o_z2 = c.take(hid), o_a2 = c.take(hid);
  const size_t o_y = c.take(out), o_dy = c.take(out), o_d1 = c.take(hid), o_d2 = c.take(hid);
  const size_t o_part = c.take(((size_t)B * MLP_OUT / 256 + 1) * 8);
  if (h) {
    h->off_p = o_p;
    h->off_g = o_g;
    h->off_m = o_m;
    h->off_v = o_v;
    h->off_z1 = o_z1;
    h->off_a1 = o_a1;
    h->off_z2 = o_z2;
    h->off_a2 = o_a2;
    h->off_y = o_y;
    h->off_dy = o_dy;
    h->off_d1 = o_d1;
    h->off_d2 = o_d2;
    h->off_part = o_part;
  }
  return c.off;
}

struct MlpParams {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
template <typename T>
void mlp_split(T* p, T*& W1, T*& b1, T*& W2, T*& b2, T*& W3, T*& b3) {
  W1 = p;
  b1 = W1 + MLP_H * MLP_IN;
  W2 = b1 + MLP_H;
  b2 = W2 + MLP_H * MLP_H;
  W3 = b2 + MLP_H;
  b3 = W3 + MLP_OUT * MLP_H;
}

dim3 gemm_grid(int M, int N) { return dim3((N + 63) / 64, (M + 63) / 64); }

// the three layers on stream st; Z1, Z2 (pre-activations, for the backward
// pass) may be null
void mlp_forward_raw(const float* prm, const float* X, int B, float* Y, float* Z1, float* A1, float* Z2,
                     float* A2, hipStream_t st) {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  mlp_split(prm, W1, b1, W2, b2, W3, b3);
  hipLaunchKernelGGL(k_gemm<EPI_BIAS_GELU>, gemm_grid(B, MLP_H), dim3(256), 0, st, X, MLP_IN, 1, W1, MLP_IN, 1, B,
                     MLP_H, MLP_IN, b1, (const float*)nullptr, Z1, A1);
  hipLaunchKernelGGL(k_gemm<EPI_BIAS_GELU>, gemm_grid(B, MLP_H), dim3(256), 0, st, (const float*)A1, MLP_H, 1, W2,
                     MLP_H, 1, B, MLP_H, MLP_H, b2, (const float*)nullptr, Z2, A2);
  hipLaunchKernelGGL(k_gemm<EPI_BIAS>, gemm_grid(B, MLP_OUT), dim3(256), 0, st, (const float*)A2, MLP_H, 1, W3,
                     MLP_H, 1, B, MLP_OUT, MLP_H, b3, (const float*)nullptr, (float*)nullptr, Y);
}

void mlp_forward(lbib_mlp* h, const float* X, int B, float* Y) {
  mlp_forward_raw(h->at<float>(h->off_p), X, B, Y, h->at<float>(h->off_z1), h->at<float>(h->off_a1),
                  h->at<float>(h->off_z2), h->at<float>(h->off_a2), h->stream);
}

// forward + loss partials + gradient into off_g
void mlp_backward(lbib_mlp* h, const float* X, const float* T, int B) {
  float *W1, *b1, *W2, *b2, *W3, *b3, *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;
  mlp_split(h->at<float>(h->off_p), W1, b1, W2, b2, W3, b3);
  mlp_split(h->at<float>(h->off_g), gW1, gb1, gW2, gb2, gW3, gb3);
  float* Y = h->at<float>(h->off_y);
  float* dY = h->at<float>(h->off_dy);
  float *Z1 = h->at<float>(h->off_z1), *A1 = h->at<float>(h->off_a1);
  float *Z2 = h->at<float>(h->off_z2), *A2 = h->at<float>(h->off_a2);
  float *D1 = h->at<float>(h->off_d1), *D2 = h->at<float>(h->off_d2);
  mlp_forward(h, X, B, Y);
  const long long n = (long long)B * MLP_OUT;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, (const float*)Y, T, n,
                     1.0f / (float)B, dY, h->at<double>(h->off_part));
  // layer 3: dW3 = dY^T A2, db3, dZ2 = (dY W3) * GELU'(Z2)
  hipLaunchKernelGGL(k_gemm<EPI_NONE>, gemm_grid(MLP_OUT, MLP_H), dim3(256), 0, h->stream, (const float*)dY, 1,
                     MLP_OUT, (const float*)A2, 1, MLP_H, MLP_OUT, MLP_H, B, (const float*)nullptr,
                     (const float*)nullptr, (float*)nullptr, gW3);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, h->stream, (const float*)dY, B, MLP_OUT, gb3);
  hipLaunchKernelGGL(k_gemm<EPI_GELU_GRAD>, gemm_grid(B, MLP_H), dim3(256), 0, h->stream, (const float*)dY,
                     MLP_OUT, 1, (const float*)W3, 1, MLP_H, B, MLP_H, MLP_OUT, (const float*)nullptr,
                     (const float*)Z2, (float*)nullptr, D2);
  // layer 2
  hipLaunchKernelGGL(k_gemm<EPI_NONE>, gemm_grid(MLP_H, MLP_H), dim3(256), 0, h->stream, (const float*)D2, 1,
                     MLP_H, (const float*)A1, 1, MLP_H, MLP_H, MLP_H, B, (const float*)nullptr,
                     (const float*)nullptr, (float*)nullptr, gW2);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, h->stream, (const float*)D2, B, MLP_H, gb2);
  hipLaunchKernelGGL(k_gemm<EPI_GELU_GRAD>, gemm_grid(B, MLP_H), dim3(256), 0, h->stream, (const float*)D2,
                     MLP_H, 1, (const float*)W2, 1, MLP_H, B, MLP_H, MLP_H, (const float*)nullptr,
                     (const float*)Z1, (float*)nullptr, D1);
  // layer 1
  hipLaunchKernelGGL(k_gemm<EPI_NONE>, gemm_grid(MLP_H, MLP_IN), dim3(256), 0, h->stream, (const float*)D1, 1,
                     MLP_H, X, 1, MLP_IN, MLP_H, MLP_IN, B, (const float*)nullptr, (const float*)nullptr,
                     (float*)nullptr, gW1);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, h->stream, (const float*)D1, B, MLP_H, gb1);
}

int mlp_loss(lbib_mlp* h, int B, double* loss) {
  const int nb = (int)(((long long)B * MLP_OUT + 255) / 256);
  std::vector<double> part(nb);
  HIPCHK(hipMemcpyAsync(part.data(), h->ws + h->off_part, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double s = 0.0;
  for (double v : part) s += v;
  *loss = 0.5 * s / B;
  return LBIB_OK;
}

}  // namespace

extern "C" {

int lbib_mlp_param_count(void) { return MLP_NPARAM; }

int lbib_mlp_workspace_bytes(int batch_max, size_t* bytes) {
  if (batch_max < 1 || batch_max > (1 << 20) || !bytes) return LBIB_EINVAL;
  *bytes = mlp_layout(nullptr, batch_max);
  return LBIB_OK;
}

int lbib_mlp_create(int batch_max, void* ws, size_t ws_bytes, void* stream, lbib_mlp** out) {
  size_t need = 0;
  int rc = lbib_mlp_workspace_bytes(batch_max, &need);
  if (rc) return rc;
  if (!ws || !out || ((uintptr_t)ws % kAlign) != 0) return LBIB_EINVAL;
  if (ws_bytes < need) return LBIB_ENOMEM;
  lbib_mlp* h = new (std::nothrow) lbib_mlp();
  if (!h) return LBIB_ENOMEM;
  h->ws = (char*)ws;
  h->stream = (hipStream_t)stream;
  h->bmax = batch_max;
  mlp_layout(h, batch_max);
  if (hipMemsetAsync(h->ws, 0, need, h->stream) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return LBIB_EHIP;
  }
  *out = h;
  return LBIB_OK;
}

int lbib_mlp_set_params(lbib_mlp* h, const float* host) {
  if (!h || !host) return LBIB_EINVAL;
  for (int k = 0; k < MLP_NPARAM; k++)
    if (!std::isfinite(host[k])) return LBIB_EINVAL;
  HIPCHK(hipMemcpyAsync(h->ws + h->off_p, host, (size_t)MLP_NPARAM * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemsetAsync(h->ws + h->off_m, 0, (size_t)MLP_NPARAM * 4, h->stream));
  HIPCHK(hipMemsetAsync(h->ws + h->off_v, 0, (size_t)MLP_NPARAM * 4, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->t = 0;
  return LBIB_OK;
}

int lbib_mlp_get_params(lbib_mlp* h, float* host) {
  if (!h || !host) return LBIB_EINVAL;
  HIPCHK(hipMemcpyAsync(host, h->ws + h->off_p, (size_t)MLP_NPARAM * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBIB_OK;
}

int lbib_mlp_forward(lbib_mlp* h, const float* x_dev, int B, float* y_dev) {
  if (!h || !x_dev || !y_dev || B < 1 || B > h->bmax) return LBIB_EINVAL;
  mlp_forward(h, x_dev, B, y_dev);
  return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
}

int lbib_mlp_gradient(lbib_mlp* h, const float* x_dev, const float* t_dev, int B, double* loss, float* grad_host) {
  if (!h || !x_dev || !t_dev || B < 1 || B > h->bmax) return LBIB_EINVAL;
  mlp_backward(h, x_dev, t_dev, B);
  if (hipGetLastError() != hipSuccess) return LBIB_EHIP;
  if (grad_host) {
    HIPCHK(hipMemcpyAsync(grad_host, h->ws + h->off_g, (size_t)MLP_NPARAM * 4, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  if (loss) return mlp_loss(h, B, loss);
  return LBIB_OK;
}

int lbib_mlp_adam_step(lbib_mlp* h, const float* x_dev, const float* t_dev, int B, float lr, float beta1,
                       float beta2, float eps, double* loss) {
  if (!h || !x_dev || !t_dev || B < 1 || B > h->bmax) return LBIB_EINVAL;
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) return LBIB_EINVAL;
  mlp_backward(h, x_dev, t_dev, B);
  h->t += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)h->t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)h->t));
  hipLaunchKernelGGL(k_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, h->stream, h->at<float>(h->off_p),
                     (const float*)h->at<float>(h->off_g), h->at<float>(h->off_m), h->at<float>(h->off_v),
                     MLP_NPARAM, lr, beta1, beta2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess) return LBIB_EHIP;
  if (loss) return mlp_loss(h, B, loss);
  return LBIB_OK;
}

void lbib_mlp_destroy(lbib_mlp* h) { delete h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// forward pass without a workspace, for callers that cannot allocate: the
// hidden activations live in a fixed device array of the library.  The
// array's name is a host-side stand-in in host code; its device address is
// looked up once per device and only that address is passed to kernels.
constexpr int MLP_NOALLOC_ROWS = 4096;
static __device__ __align__(256) float scratch[2 * MLP_NOALLOC_ROWS * MLP_H];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};  // device address of scratch, per device

// address of the current device's scratch (looked up on the first call made
// with that device current)
int scratch_address(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBIB_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return LBIB_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBIB_EHIP;
    g_scratch[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch[dev];
  return LBIB_OK;
}
}  // namespace

extern "C" int lbib_mlp_forward_noalloc(const float* params_dev, const float* x_dev, int B, float* y_dev,
                                        void* hip_stream) {
  if (!params_dev || !x_dev || !y_dev || B < 1) return LBIB_EINVAL;
  if (B > MLP_NOALLOC_ROWS) return LBIB_ENOMEM;
  float* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc) return rc;
  // A1 and A2 are written in full before they are read: nothing to clear
  float* A1 = base;
  float* A2 = base + (size_t)MLP_NOALLOC_ROWS * MLP_H;
  mlp_forward_raw(params_dev, x_dev, B, y_dev, nullptr, A1, nullptr, A2, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? LBIB_OK : LBIB_EHIP;
}
