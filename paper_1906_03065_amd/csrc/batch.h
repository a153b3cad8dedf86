// batch.h -- many independent D2Q9 simulations stepped together.
//
// Every phase of the step runs as one launch over all members: the grid
// walks a queue of work items (a membrane, an active tile, a marker, a
// (strip, segment) of a lattice) spread over the members, finds the member
// of each item by binary search over prefix sums, and runs the same device
// code the single-simulation kernels run.  The lattice kernel runs once per
// size class, since the strip width (lanes per workgroup) is chosen per
// class, with one (strip, segment) item per workgroup.  All members advance
// with the same buffer parity.
#pragma once
#include "common.h"
#include "k_ibm.h"
#include "k_lb.h"

namespace lb {

constexpr int BATCH_MAX = 256;  // members per batch

template <class St>
struct BMember {
  LBParams P;  // strips and segments for the member's size class
  St a, b;     // population buffers (parity 0 reads a, writes b)
  MemDev md;
  TileMap tm;
  CoupArgs ca;
  double* Ifield;
  long long* fib;
  double* force;
};

// The member descriptors live in global memory; every kernel copies the one
// it works on into registers first, so the stores of the step cannot be
// taken to alias it (which would force a reload after each store).

// index i in [0, n) with pre[i] <= v < pre[i + 1]
__device__ __forceinline__ int prefix_find(const int* pre, int n, int v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <class St>
__global__ void kb_begin(BMember<St>* T, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    int* ts = T[i].tm.tstate;
    ts[0] = 0;
    ts[1] = ts[1] + 1;
  }
}

// one workgroup per (member, membrane)
template <class St, int NT>
__global__ __launch_bounds__(NT) void kb_tiles(const BMember<St>* T, const int2* mems) {
  const int2 e = mems[blockIdx.x];
  const MemDev md = T[e.x].md;
  const TileMap tm = T[e.x].tm;
  const LBParams P = T[e.x].P;
  const double rc = T[e.x].ca.r_cut;
  tiles_run<NT>(md, tm, P.nx, P.ny, 1, P.wall_y, 0, 2, map_reach(rc), e.y, tm.tstate[1], tm.tstate);
}

// persistent: the active tiles of all members
template <class St, typename R, int NT>
__global__ __launch_bounds__(NT, 2) void kb_coupling2d(const BMember<St>* T, int n, int parity) {
  __shared__ int s_pre[BATCH_MAX + 1];
  for (int i = threadIdx.x; i < n; i += NT) s_pre[i + 1] = T[i].tm.tstate[0];
  if (threadIdx.x == 0) s_pre[0] = 0;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 0; i < n; i++) s_pre[i + 1] += s_pre[i];
  __syncthreads();
  const int total = s_pre[n];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int i = prefix_find(s_pre, n, item);
    const MemDev md = T[i].md;
    const TileMap tm = T[i].tm;
    const CoupArgs ca = T[i].ca;
    double* Ifield = T[i].Ifield;
    const St cur = parity ? T[i].b : T[i].a;
    coupling2d_tile<St, R, NT>(md, tm, ca, Ifield, cur, item - s_pre[i]);
  }
}

// markers of all members (mpre: marker prefix, n + 1 entries)
template <class St>
__global__ void kb_forcespread2d(const BMember<St>* T, const int* __restrict__ mpre, int n) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gf = tid >> 4, k = tid & 15;
  const bool live = gf < mpre[n];
  const int i = live ? prefix_find(mpre, n, gf) : 0;
  const MemDev md = T[i].md;
  long long* fib = T[i].fib;
  const int nx = T[i].P.nx, ny = T[i].P.ny, wy = T[i].P.wall_y;
  forcespread2d_run(md, fib, nx, ny, wy, live ? gf - mpre[i] : 0, k, live);
}

template <class St, typename R>
__global__ void kb_interp2d(const BMember<St>* T, const int* __restrict__ mpre, int n, int parity) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int gf = tid >> 4, k = tid & 15;
  const bool live = gf < mpre[n];
  const int i = live ? prefix_find(mpre, n, gf) : 0;
  const MemDev md = T[i].md;
  const LBParams P = T[i].P;
  const double* force = T[i].force;
  // after the lattice update the current state is in the buffer written
  const St cur = parity ? T[i].a : T[i].b;
  interp2d_run<St, R>(md, cur, P, force, live ? gf - mpre[i] : 0, k, live);
}

// one workgroup per (strip, segment) item of the members of one size class
// (cm: their member ids, bpre: item prefix, ncm + 1 entries)
template <class St, typename R, int BX, int NS, int WPE, int FORM = 0>
__global__ __launch_bounds__(BX, WPE) void kb_lb2d(const BMember<St>* T, const int* __restrict__ cm,
                                                   const int* __restrict__ bpre, int ncm, int parity) {
  // one work item per workgroup: without a loop over items the kernel
  // fits the single kernel's register budget (three waves per SIMD)
  const int total = bpre[ncm];
  {
    if ((int)blockIdx.x >= total) return;
    // items dealt to the eight XCDs in contiguous runs, so the neighbouring
    // segments of a member share their halo rows in one L2
    const int item = (int)gridDim.x == total ? dealt_index((int)blockIdx.x, total, 8) : (int)blockIdx.x;
    const int q = prefix_find(bpre, ncm, item);
    const int i = cm[q];
    const LBParams P = T[i].P;
    const St src = parity ? T[i].b : T[i].a, dst = parity ? T[i].a : T[i].b;
    const int* tflag = T[i].tm.tflag;
    const int* tstate = T[i].tm.tstate;
    const double* Ifield = T[i].Ifield;
    long long* fib = T[i].fib;
    double* force = T[i].force;
    int strip, sgm;
    strip_segment(item - bpre[q], P.nstrip, P.nseg, 1, strip, sgm);
    const int y0 = sgm * P.seg, y1 = min(y0 + P.seg, P.ny);
    lb2d_run<St, R, BX, NS, FORM>(src, dst, P, strip, y0, y1, (sgm & 1) ? -1 : 1, tflag, tstate, Ifield, fib,
                                  force);
  }
}

}  // namespace lb
