/*
 * orc.c -- plain FP64 CPU oracle of the ternary free-energy LB + IBM step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.  Loops are written in the order the paper states
 * the method; OpenMP only splits independent per-node loops, every sum over
 * nodes or markers runs serially in a fixed order.
 *
 * Paper sections followed (Pepona et al.):
 *   Sec. 2.1  eq. MassDensity                        component densities (the
 *             extension Sec. 5 names; all 1 in the paper's model)
 *   Sec. 2.5  eq. LandauFE, CouplingE, Iprofile     free energy, coupling profile
 *   Sec. 2.6  eq. VariableTransform                  rho, phi, psi from C_m
 *   Sec. 3.1  eq. LBE, EDF, MomentsDFs, ActualFluidVel, VelCorrection,
 *             ForceFE, GradPT                        lattice Boltzmann step
 *   Sec. 3.2  eq. DiscreteSE..DiscreteTF              membrane energies / forces
 *   Sec. 3.3  eq. Spreading, DiscreteDirac, Interpolation, UpdatedXl
 *   App. A    eq. AppA                                chemical potentials
 * Readings where the paper is silent are marked READING in the comments.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#include <complex.h>
#undef I /* complex.h's imaginary unit; written _Complex_I below */
#endif

#define MAXQ 19
#define MAXMEM 1024
#define CS2 (1.0 / 3.0)

typedef struct {
  int Q, D;
  int c[MAXQ][3];
  double w[MAXQ];
  int opp[MAXQ];
} lat_t;

typedef struct {
  int n;          /* markers                                   */
  int ntri;       /* 3D triangles (0 in 2D)                     */
  int nedge;      /* 2D: n segments l -> l+1; 3D: mesh edges    */
  double* X;      /* 3 per marker                               */
  double* U;      /* 3 per marker: last interpolated velocity   */
  double* F;      /* 3 per marker: last total force             */
  double* rest;   /* rest length per segment / edge             */
  int* tri;       /* 3 per triangle                             */
  int* edge;      /* 2 per edge (3D)                            */
  int* etri;      /* 2 per edge: the adjacent triangles (3D)    */
  double ks, kb;
  int law;        /* strain law (orc_set_membrane_law)                */
} mem_t;

struct orc_sim {
  orc_params p;
  lat_t L;
  int D, nx, ny, nz;
  long N;
  double* pop[3];   /* f, g, h: [Q][N], populations at the current time  */
  double* nxt[3];   /* stream targets                                    */
  double *rho, *u, *phi, *psi;  /* moments; u has 3 per node            */
  double* I;        /* coupling profile, eq. Iprofile                    */
  double* mu[3];    /* mu_rho (no ideal-gas part), mu_phi, mu_psi'       */
  double* lap[3];
  double* grad;     /* scratch 3 per node                                */
  double* force;    /* total force f of the last step, 3 per node        */
  double* fib;      /* spread membrane force, 3 per node                 */
  double* sd;       /* scratch: signed distance per node                 */
  int* seg;         /* scratch: closest element per node (-1: none)      */
  double* bary;     /* scratch: 3 weights per node                       */
  double* foot;     /* scratch: closest point, 3 per node                */
  mem_t mem[MAXMEM];
  int nmem;
  long steps;
  int ready;
};

/* ------------------------------------------------------------------ */
/* lattices                                                            */
/* ------------------------------------------------------------------ */
static int lat_make(int kind, lat_t* L) {
  memset(L, 0, sizeof *L);
  if (kind == 0) {
    /* D2Q9 velocity set and weights of Sec. 3.1, in the order printed there */
    static const int cx[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
    static const int cy[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
    L->Q = 9;
    L->D = 2;
    for (int i = 0; i < 9; i++) {
      L->c[i][0] = cx[i];
      L->c[i][1] = cy[i];
      L->w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
  } else if (kind == 1) {
    /* D3Q19 (the paper states the 3D extension is direct): rest particle,
       six face neighbours, twelve edge neighbours */
    L->Q = 19;
    L->D = 3;
    int q = 0;
    L->w[q++] = 1.0 / 3.0;
    for (int a = 0; a < 3; a++)
      for (int sgn = 1; sgn >= -1; sgn -= 2) {
        L->c[q][a] = sgn;
        L->w[q++] = 1.0 / 18.0;
      }
    for (int a = 0; a < 3; a++)
      for (int b = a + 1; b < 3; b++)
        for (int sa = 1; sa >= -1; sa -= 2)
          for (int sb = 1; sb >= -1; sb -= 2) {
            L->c[q][a] = sa;
            L->c[q][b] = sb;
            L->w[q++] = 1.0 / 36.0;
          }
  } else {
    return -1;
  }
  for (int i = 0; i < L->Q; i++)
    for (int j = 0; j < L->Q; j++)
      if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
        L->opp[i] = j;
  return 0;
}

int orc_lattice(int lattice, int* Q, int* c, double* w) {
  lat_t L;
  if (lat_make(lattice, &L)) return -1;
  *Q = L.Q;
  for (int i = 0; i < L.Q; i++) {
    for (int a = 0; a < 3; a++) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* equilibria, eq. EDF                                                 */
/* ------------------------------------------------------------------ */
static void feq_all(const lat_t* L, double rho, const double* u, double* out) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L->Q; i++) {
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    out[i] = L->w[i] * rho * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2));
  }
}

/* g^eq / h^eq: moving populations from the formula, rest population fixed by
   the zeroth moment (q minus the sum of the others) */
static void geq_all(const lat_t* L, double q, double mu, double Gamma, const double* v, double* out) {
  double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  double rest = q;
  for (int i = 1; i < L->Q; i++) {
    double cv = L->c[i][0] * v[0] + L->c[i][1] * v[1] + L->c[i][2] * v[2];
    out[i] = L->w[i] * (Gamma * mu / CS2 + q * cv / CS2 + q * (cv * cv - CS2 * vv) / (2.0 * CS2 * CS2));
    rest -= out[i];
  }
  out[0] = rest;
}

int orc_feq(int lattice, double rho, const double* u, double* out) {
  lat_t L;
  if (lat_make(lattice, &L)) return -1;
  double uu[3] = {u[0], u[1], L.D == 3 ? u[2] : 0.0};
  feq_all(&L, rho, uu, out);
  return 0;
}

int orc_geq(int lattice, double q, double mu, double Gamma, const double* v, double* out) {
  lat_t L;
  if (lat_make(lattice, &L)) return -1;
  double vv[3] = {v[0], v[1], L.D == 3 ? v[2] : 0.0};
  geq_all(&L, q, mu, Gamma, vv, out);
  return 0;
}

/* ------------------------------------------------------------------ */
/* chemical potentials, Appendix A.                                    */
/* READING: the ideal-gas part c_s^2 (ln rho + 1) of mu_rho is left out; its   */
/* gradient term cancels the divergence of rho c_s^2 I in eq. ForceFE, so the  */
/* thermodynamic force is -rho grad mu_rho - phi grad mu_phi - psi grad mu_psi'.*/
/* mu_psi' adds the coupling term kappa_c (psi - I) (Sec. 3.1).                 */
/* ------------------------------------------------------------------ */
/* ------------------------------------------------------------------ */
/* Unequal component densities (the extension named in Sec. 5): eq.     */
/* MassDensity makes the LB density the mass density rho = sum M_m C_m  */
/* while phi = C1 - C2 and psi = C3 stay as in eq. VariableTransform.    */
/* READING: the concentrations then follow linearly from (rho, phi, psi) */
/* with n = C1 + C2 + C3 = (rho - a phi - b psi) / Mb, Mb = (M1 + M2)/2, */
/* a = (M1 - M2)/2, b = M3 - Mb; the Landau energy keeps its form in the */
/* C_m; the ideal gas is that of n, c_s^2 Mb n ln n, so the LB carries  */
/* the pressure p0 = c_s^2 Mb n: its equilibrium adds 3 w_i dp (i > 0,   */
/* -3 (1 - w_0) dp at rest) to f_i^eq with dp = p0 - c_s^2 rho, and in  */
/* each bulk phase (n = 1) p0 is the same whatever its density.  All     */
/* M_m = 1 gives the paper's model exactly.                              */
/* ------------------------------------------------------------------ */
static void mw_get(const orc_params* p, double M[3]) {
  for (int m = 0; m < 3; m++) M[m] = p->mw[m] > 0.0 ? p->mw[m] : 1.0;
}

static int equal_densities(const orc_params* p) {
  double M[3];
  mw_get(p, M);
  return M[0] == 1.0 && M[1] == 1.0 && M[2] == 1.0;
}

/* A[m][q]: dC_m / d(rho, phi, psi)_q */
static void conc_matrix(const orc_params* p, double A[3][3]) {
  double M[3];
  mw_get(p, M);
  const double Mb = 0.5 * (M[0] + M[1]), a = 0.5 * (M[0] - M[1]), b = M[2] - Mb;
  A[0][0] = 0.5 / Mb;  A[0][1] = 0.5 * (1.0 - a / Mb);  A[0][2] = 0.5 * (-1.0 - b / Mb);
  A[1][0] = 0.5 / Mb;  A[1][1] = 0.5 * (-1.0 - a / Mb); A[1][2] = 0.5 * (-1.0 - b / Mb);
  A[2][0] = 0.0;       A[2][1] = 0.0;                    A[2][2] = 1.0;
}

void orc_concentrations(const orc_params* p, double rho, double phi, double psi, double* C) {
  if (equal_densities(p)) {
    /* eq. VariableTransform inverted */
    C[0] = 0.5 * (rho + phi - psi);
    C[1] = 0.5 * (rho - phi - psi);
    C[2] = psi;
    return;
  }
  double A[3][3];
  conc_matrix(p, A);
  const double q[3] = {rho, phi, psi};
  for (int m = 0; m < 3; m++) C[m] = A[m][0] * q[0] + A[m][1] * q[1] + A[m][2] * q[2];
}

/* the LB pressure shift dp = p0 - c_s^2 rho = -c_s^2 (a phi + b psi) */
static double pressure_shift(const orc_params* p, double phi, double psi) {
  double M[3];
  mw_get(p, M);
  const double Mb = 0.5 * (M[0] + M[1]), a = 0.5 * (M[0] - M[1]), b = M[2] - Mb;
  return -CS2 * (a * phi + b * psi);
}

/* with component densities: the shift of f_i^eq that makes the lattice's
   pressure p0 instead of c_s^2 rho (zero for equal densities) */
static void feq_pressure_shift(const lat_t* L, const orc_params* p, double phi, double psi, double* sh) {
  const double dp = equal_densities(p) ? 0.0 : pressure_shift(p, phi, psi);
  for (int i = 0; i < L->Q; i++) sh[i] = (i == 0 ? -(1.0 - L->w[0]) : L->w[i]) * dp / CS2;
}

/* mu_q = sum_m (dC_m/dq) dF/dC_m, dF/dC_m = kappa_m C (1 - C)(1 - 2C) -
   alpha^2 kappa_m lap C_m, lap C_m = sum_q (dC_m/dq) lap q; the coupling
   term kappa_c (psi - I) joins mu_psi */
void orc_mu_general(const orc_params* p, double rho, double phi, double psi, double lr, double lp,
                    double ls, double I, double* mu3) {
  double A[3][3];
  conc_matrix(p, A);
  const double q[3] = {rho, phi, psi}, l[3] = {lr, lp, ls};
  const double km[3] = {p->kappa1, p->kappa2, p->kappa3}, a2 = p->alpha * p->alpha;
  double bm[3];
  for (int m = 0; m < 3; m++) {
    double C = 0.0, L = 0.0;
    for (int k = 0; k < 3; k++) {
      C += A[m][k] * q[k];
      L += A[m][k] * l[k];
    }
    bm[m] = km[m] * C * (1.0 - C) * (1.0 - 2.0 * C) - a2 * km[m] * L;
  }
  for (int k = 0; k < 3; k++) mu3[k] = A[0][k] * bm[0] + A[1][k] * bm[1] + A[2][k] * bm[2];
  mu3[2] += p->kappa_c * (psi - I);
}

void orc_mu(const orc_params* p, double rho, double phi, double psi, double lr, double lp,
            double ls, double I, double* mu3) {
  if (!equal_densities(p)) {
    orc_mu_general(p, rho, phi, psi, lr, lp, ls, I, mu3);
    return;
  }
  const double k1 = p->kappa1, k2 = p->kappa2, k3 = p->kappa3, a2 = p->alpha * p->alpha;
  const double x = rho + phi - psi; /* 2 C1 */
  const double y = rho - phi - psi; /* 2 C2 */
  const double tx = k1 / 8.0 * x * (x - 1.0) * (x - 2.0);
  const double ty = k2 / 8.0 * y * (y - 1.0) * (y - 2.0);
  mu3[0] = tx + ty + a2 / 4.0 * ((k1 + k2) * (ls - lr) + (k2 - k1) * lp);
  mu3[1] = tx - ty + a2 / 4.0 * ((k2 - k1) * (lr - ls) - (k1 + k2) * lp);
  mu3[2] = -tx - ty + a2 / 4.0 * ((k1 + k2) * lr - (k2 - k1) * lp - (k1 + k2 + 4.0 * k3) * ls) +
           k3 * psi * (psi - 1.0) * (2.0 * psi - 1.0) + p->kappa_c * (psi - I);
}

/* ------------------------------------------------------------------ */
/* lattice geometry helpers                                            */
/* ------------------------------------------------------------------ */
static inline long nid(const orc_sim* s, int x, int y, int z) {
  return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}

static inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

/* neighbour for finite differences: periodic wrap, or mirror ghost across a
   wall at -1/2 and n-1/2 (READING: zero normal gradient at walls, eq. NaturalBCs) */
static inline int fd_coord(int v, int n, int wall) {
  if (!wall) return wrapi(v, n);
  if (v < 0) return -1 - v;
  if (v >= n) return 2 * n - 1 - v;
  return v;
}

static inline long fd_nbr(const orc_sim* s, int x, int y, int z, int i) {
  const lat_t* L = &s->L;
  int xx = wrapi(x + L->c[i][0], s->nx);
  int yy = fd_coord(y + L->c[i][1], s->ny, s->p.wall_y);
  int zz = (s->D == 3) ? fd_coord(z + L->c[i][2], s->nz, s->p.wall_z) : 0;
  return nid(s, xx, yy, zz);
}

/* streaming target, or -1 when the link crosses a wall */
static inline long stream_dest(const orc_sim* s, int x, int y, int z, int i) {
  const lat_t* L = &s->L;
  int xx = wrapi(x + L->c[i][0], s->nx);
  int yy = y + L->c[i][1];
  if (s->p.wall_y) {
    if (yy < 0 || yy >= s->ny) return -1;
  } else {
    yy = wrapi(yy, s->ny);
  }
  int zz = 0;
  if (s->D == 3) {
    zz = z + L->c[i][2];
    if (s->p.wall_z) {
      if (zz < 0 || zz >= s->nz) return -1;
    } else {
      zz = wrapi(zz, s->nz);
    }
  }
  return nid(s, xx, yy, zz);
}

/* ------------------------------------------------------------------ */
/* isotropic stencils: grad q = (1/c_s^2) sum w_i c_i q(x+c_i),        */
/* lap q = (2/c_s^2) sum w_i (q(x+c_i) - q(x)).  READING: the paper     */
/* does not print its stencils; these are the standard lattice ones.    */
/* ------------------------------------------------------------------ */
int orc_grad_lap(const orc_sim* s, const double* q, double* grad, double* lap) {
  const lat_t* L = &s->L;
  const int D = s->D;
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < s->nz; z++)
    for (int y = 0; y < s->ny; y++)
      for (int x = 0; x < s->nx; x++) {
        long n = nid(s, x, y, z);
        double g[3] = {0, 0, 0}, l = 0.0;
        for (int i = 0; i < L->Q; i++) {
          double qn = q[fd_nbr(s, x, y, z, i)];
          for (int a = 0; a < 3; a++) g[a] += L->w[i] * L->c[i][a] * qn;
          l += L->w[i] * (qn - q[n]);
        }
        if (grad)
          for (int a = 0; a < D; a++) grad[n * D + a] = g[a] / CS2;
        if (lap) lap[n] = 2.0 * l / CS2;
      }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Peskin four-point kernel, eq. DiscreteDirac                         */
/* ------------------------------------------------------------------ */
double orc_peskin(double r) {
  double a = fabs(r);
  if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
  return 0.0;
}

/* visit the 4^d stencil nodes of a marker at X: callback gets node index and
   weight delta_h(x - X).  Nodes beyond a wall are skipped (READING: the paper
   has periodic boundaries only). */
typedef void (*stencil_fn)(void* ctx, long node, double wgt);
static void stencil_visit(const orc_sim* s, const double* X, stencil_fn fn, void* ctx) {
  int base[3] = {0, 0, 0};
  for (int a = 0; a < s->D; a++) base[a] = (int)floor(X[a]) - 1;
  int kz_n = (s->D == 3) ? 4 : 1;
  for (int kz = 0; kz < kz_n; kz++)
    for (int ky = 0; ky < 4; ky++)
      for (int kx = 0; kx < 4; kx++) {
        int cx = base[0] + kx, cy = base[1] + ky, cz = base[2] + kz;
        double wgt = orc_peskin(cx - X[0]) * orc_peskin(cy - X[1]);
        if (s->D == 3) wgt *= orc_peskin(cz - X[2]);
        int yy, zz = 0;
        if (s->p.wall_y) {
          if (cy < 0 || cy >= s->ny) continue;
          yy = cy;
        } else {
          yy = wrapi(cy, s->ny);
        }
        if (s->D == 3) {
          if (s->p.wall_z) {
            if (cz < 0 || cz >= s->nz) continue;
            zz = cz;
          } else {
            zz = wrapi(cz, s->nz);
          }
        }
        fn(ctx, nid(s, wrapi(cx, s->nx), yy, zz), wgt);
      }
}

typedef struct { double* out; const double* F; int D; } spread_ctx;
static void spread_cb(void* c, long node, double wgt) {
  spread_ctx* k = (spread_ctx*)c;
  for (int a = 0; a < k->D; a++) k->out[node * k->D + a] += k->F[a] * wgt;
}

/* eq. Spreading.  READING: marker forces are spread without the extra Delta s
   factor (it is 1 in the paper's setup); this keeps the spread total equal to
   the sum of marker forces. */
int orc_spread(const orc_sim* s, int n, const double* X, const double* F, double* fib) {
  const int D = s->D;
  memset(fib, 0, sizeof(double) * (size_t)s->N * D);
  for (int l = 0; l < n; l++) {
    spread_ctx k = {fib, F + (size_t)l * D, D};
    stencil_visit(s, X + (size_t)l * D, spread_cb, &k);
  }
  return 0;
}

typedef struct { const double* v; double acc[3]; int D; } interp_ctx;
static void interp_cb(void* c, long node, double wgt) {
  interp_ctx* k = (interp_ctx*)c;
  for (int a = 0; a < k->D; a++) k->acc[a] += k->v[node * k->D + a] * wgt;
}

/* eq. Interpolation (delta x = 1) */
int orc_interp(const orc_sim* s, int n, const double* X, const double* v, double* U) {
  const int D = s->D;
  for (int l = 0; l < n; l++) {
    interp_ctx k = {v, {0, 0, 0}, D};
    stencil_visit(s, X + (size_t)l * D, interp_cb, &k);
    for (int a = 0; a < D; a++) U[(size_t)l * D + a] = k.acc[a];
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* 2D ring membrane, eqs. DiscreteSE, DiscreteBE, DiscreteTheta,       */
/* DiscreteArcLength, DiscreteSF, DiscreteBF.                          */
/* Markers l = 0..n-1 form a closed ring; segment l joins l and l+1.   */
/* ------------------------------------------------------------------ */
/* Strain energy per unit rest length of a segment stretched by lam, and its
   derivative dW/dlam (the segment's tension).  law 0: eq. DiscreteSE,
   ks/2 (lam - 1)^2.  Laws 1 and 2 (READING: the paper names neo-Hookean and
   Skalak membranes without formulas): the membrane laws per unit reference
   area with the second principal stretch fixed at 1 (a 2D ring is the
   section of a membrane under plane strain), scaled to the same small-strain
   modulus ks:
     neo-Hookean  G/2 (l1^2 + l2^2 + 1/(l1 l2)^2 - 3), G = ks/4
                  -> ks/8 (lam - 1/lam)^2
     Skalak       G/4 (I1^2 + 2 I1 - 2 I2 + C I2^2), I1 = l1^2 + l2^2 - 2,
                  I2 = (l1 l2)^2 - 1, G (1 + C) = ks/2
                  -> ks/8 (lam^2 - 1)^2 (C only scales it at plane strain) */
static void strain_law(int law, double ks, double lam, double* W, double* T) {
  if (law == 1) {
    double q = lam - 1.0 / lam;
    *W = ks / 8.0 * q * q;
    *T = ks / 4.0 * q * (1.0 + 1.0 / (lam * lam));
  } else if (law == 2) {
    double q = lam * lam - 1.0;
    *W = ks / 8.0 * q * q;
    *T = ks / 2.0 * q * lam;
  } else {
    double q = lam - 1.0;
    *W = 0.5 * ks * q * q;
    *T = ks * q;
  }
}

int orc_ring_forces(int n, const double* X, const double* rest, double ks, double kb, double* F,
                    double* E_s, double* E_b) {
  return orc_ring_forces_law(n, X, rest, ks, kb, 0, F, E_s, E_b);
}

int orc_ring_forces_law(int n, const double* X, const double* rest, double ks, double kb, int law,
                        double* F, double* E_s, double* E_b) {
  if (n < 3 || law < 0 || law > 2) return -1;
  double es = 0.0, eb = 0.0;
  for (int l = 0; l < 2 * n; l++) F[l] = 0.0;
  /* strain: E_s = sum_l W(len_l/ds_l) ds_l */
  for (int l = 0; l < n; l++) {
    int m = (l + 1) % n;
    double dx = X[2 * m] - X[2 * l], dy = X[2 * m + 1] - X[2 * l + 1];
    double len = sqrt(dx * dx + dy * dy);
    double ds = rest[l];
    double W, T;
    strain_law(law, ks, len / ds, &W, &T);
    es += W * ds;
    /* dE/dX_m = T e_l, dE/dX_l = -T e_l (e_l the unit vector l -> m) */
    double gx = T * dx / len, gy = T * dy / len;
    F[2 * m] -= gx;
    F[2 * m + 1] -= gy;
    F[2 * l] += gx;
    F[2 * l + 1] += gy;
  }
  /* bending: E_b = kb/4 sum (dtheta)^2 / ds', dtheta = 2 arccos y; the turning
     angle theta at a marker is taken from atan2(cross, dot) of the incoming
     segment b = X_l - X_{l-1} and the outgoing one a = X_{l+1} - X_l, which is
     arccos y with a well-conditioned derivative. */
  for (int l = 0; l < n; l++) {
    int lp = (l + 1) % n, lm = (l + n - 1) % n;
    double ax = X[2 * lp] - X[2 * l], ay = X[2 * lp + 1] - X[2 * l + 1];
    double bx = X[2 * l] - X[2 * lm], by = X[2 * l + 1] - X[2 * lm + 1];
    double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by);
    double cr = ax * by - ay * bx; /* a x b */
    double dt = ax * bx + ay * by; /* a . b */
    double th = atan2(cr, dt);     /* signed; theta^2 = arccos(y)^2 */
    double L = la + lb;
    eb += kb * th * th / L;        /* kb/4 (2 theta)^2 / L */
    /* d theta/da and d theta/db for theta = atan2(a x b, a . b) */
    double den = la * la * lb * lb;
    double dth_ax = (dt * by - cr * bx) / den, dth_ay = (dt * (-bx) - cr * by) / den;
    double dth_bx = (dt * (-ay) - cr * ax) / den, dth_by = (dt * ax - cr * ay) / den;
    /* e = kb th^2 / L; de/da = kb (2 th dth/da / L - th^2/L^2 a/|a|) */
    double ga_x = kb * (2.0 * th * dth_ax / L - th * th / (L * L) * ax / la);
    double ga_y = kb * (2.0 * th * dth_ay / L - th * th / (L * L) * ay / la);
    double gb_x = kb * (2.0 * th * dth_bx / L - th * th / (L * L) * bx / lb);
    double gb_y = kb * (2.0 * th * dth_by / L - th * th / (L * L) * by / lb);
    /* a = X_{l+1} - X_l, b = X_l - X_{l-1}; F = -dE/dX */
    F[2 * lp] -= ga_x;
    F[2 * lp + 1] -= ga_y;
    F[2 * l] += ga_x - gb_x;
    F[2 * l + 1] += ga_y - gb_y;
    F[2 * lm] += gb_x;
    F[2 * lm + 1] += gb_y;
  }
  if (E_s) *E_s = es;
  if (E_b) *E_b = eb;
  return 0;
}

/* ------------------------------------------------------------------ */
/* 3D closed triangle mesh.  READING (the paper's membrane law is 2D):  */
/* edge springs E_s = ks/2 sum (len/len0 - 1)^2 len0, the 3D analogue  */
/* of eq. DiscreteSE, and dihedral bending E_b = kb sum_e (1 - cos th_e)*/
/* with th_e the angle between the normals of the two triangles on e   */
/* (flat rest angle, like the zero spontaneous curvature in 2D).       */
/* ------------------------------------------------------------------ */
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* build the edge list of a closed mesh with the two triangles of each edge */
static int mesh_edges(int n, int ntri, const int* tri, int** edge_out, int** etri_out) {
  int cap = 3 * ntri;
  int* e = (int*)malloc(sizeof(int) * 2 * cap);
  int* et = (int*)malloc(sizeof(int) * 2 * cap);
  int ne = 0;
  for (int t = 0; t < ntri; t++)
    for (int k = 0; k < 3; k++) {
      int a = tri[3 * t + k], b = tri[3 * t + (k + 1) % 3];
      if (a < 0 || a >= n || b < 0 || b >= n) { free(e); free(et); return -1; }
      int lo = a < b ? a : b, hi = a < b ? b : a, found = -1;
      for (int j = 0; j < ne; j++)
        if (e[2 * j] == lo && e[2 * j + 1] == hi) { found = j; break; }
      if (found < 0) {
        e[2 * ne] = lo;
        e[2 * ne + 1] = hi;
        et[2 * ne] = t;
        et[2 * ne + 1] = -1;
        ne++;
      } else {
        if (et[2 * found + 1] != -1) { free(e); free(et); return -2; }
        et[2 * found + 1] = t;
      }
    }
  for (int j = 0; j < ne; j++)
    if (et[2 * j + 1] < 0) { free(e); free(et); return -3; } /* open mesh */
  *edge_out = e;
  *etri_out = et;
  return ne;
}

/* unnormalised normal of triangle t and its gradient contribution helper */
static void tri_normal(const double* X, const int* tri, int t, double* nrm) {
  const double *p0 = X + 3 * tri[3 * t], *p1 = X + 3 * tri[3 * t + 1], *p2 = X + 3 * tri[3 * t + 2];
  double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  cross3(e1, e2, nrm);
}

/* add to G (3 per vertex) the gradient of s(n) where n = (p1-p0)x(p2-p0) is
   triangle t's area vector and dn gives ds/dn */
static void add_normal_grad(const double* X, const int* tri, int t, const double* dsdn, double* G) {
  int v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
  const double *p0 = X + 3 * v0, *p1 = X + 3 * v1, *p2 = X + 3 * v2;
  double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
  /* n = e1 x e2; dn = de1 x e2 + e1 x de2; ds = dsdn . dn
     ds/de1 = e2 x dsdn, ds/de2 = dsdn x e1 */
  double g1[3], g2[3];
  cross3(e2, dsdn, g1);
  cross3(dsdn, e1, g2);
  for (int a = 0; a < 3; a++) {
    G[3 * v1 + a] += g1[a];
    G[3 * v2 + a] += g2[a];
    G[3 * v0 + a] -= g1[a] + g2[a];
  }
}

/* Hyperelastic triangle laws of a 3D mesh (READING: the paper names
   neo-Hookean and Skalak membranes as alternatives, without formulas).  A
   flat triangle maps linearly from its rest shape (given by the rest lengths
   a_k of the edges opposite its vertices k) to its current shape, with right
   Cauchy-Green invariants I1 = l1^2 + l2^2 = sum_k cot(theta_k) / (2 A0)
   |edge_k|^2 (theta_k the rest angle at vertex k, edge_k the current edge
   opposite it) and J = l1 l2 = A / A0.  Energy per rest area, shear modulus G = ks:
     law 1 neo-Hookean  G/2 (I1 + 1/J^2 - 3)
     law 2 Skalak       G/4 ((I1-2)^2 + 2 (I1-2) - 2 (J^2-1) + C (J^2-1)^2), C = 1
   The triangle's energy is A0 W.  Evaluated in complex arithmetic so that
   its derivatives come from the complex step (exact to round-off). */
static double complex tri_law_energy(int law, double G, const double complex* P[3], const double a[3]) {
  const double a2[3] = {a[0] * a[0], a[1] * a[1], a[2] * a[2]};
  const double A0 = 0.25 * sqrt(2.0 * (a2[0] * a2[1] + a2[1] * a2[2] + a2[2] * a2[0]) - a2[0] * a2[0] -
                                a2[1] * a2[1] - a2[2] * a2[2]);
  double complex I1 = 0.0;
  for (int k = 0; k < 3; k++) {
    const double complex* u = P[(k + 1) % 3];
    const double complex* v = P[(k + 2) % 3];
    double complex l2 = 0.0;
    for (int d = 0; d < 3; d++) l2 += (v[d] - u[d]) * (v[d] - u[d]);
    const double cot = (a2[(k + 1) % 3] + a2[(k + 2) % 3] - a2[k]) / (4.0 * A0);
    I1 += cot / (2.0 * A0) * l2;
  }
  double complex e1[3], e2[3];
  for (int d = 0; d < 3; d++) {
    e1[d] = P[1][d] - P[0][d];
    e2[d] = P[2][d] - P[0][d];
  }
  const double complex nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                       nz = e1[0] * e2[1] - e1[1] * e2[0];
  const double complex J = 0.5 * csqrt(nx * nx + ny * ny + nz * nz) / A0;
  double complex W;
  if (law == 1) {
    W = 0.5 * G * (I1 + 1.0 / (J * J) - 3.0);
  } else {
    const double complex i1 = I1 - 2.0, k2 = J * J - 1.0;
    W = 0.25 * G * (i1 * i1 + 2.0 * i1 - 2.0 * k2 + 1.0 * k2 * k2);
  }
  return A0 * W;
}

int orc_mesh_forces(int n, const double* X, int ntri, const int* tri, const double* rest_edge,
                    double ks, double kb, double* F, double* E_s, double* E_b) {
  return orc_mesh_forces_law(n, X, ntri, tri, rest_edge, ks, kb, 0, F, E_s, E_b);
}

int orc_mesh_forces_law(int n, const double* X, int ntri, const int* tri, const double* rest_edge,
                        double ks, double kb, int law, double* F, double* E_s, double* E_b) {
  if (law < 0 || law > 2) return -1;
  int *edge = NULL, *etri = NULL;
  int ne = mesh_edges(n, ntri, tri, &edge, &etri);
  if (ne < 0) return -1;
  double* G = (double*)calloc((size_t)3 * n, sizeof(double)); /* dE/dX */
  double es = 0.0, eb = 0.0;
  for (int j = 0; j < ne; j++) {
    int a = edge[2 * j], b = edge[2 * j + 1];
    double d[3] = {X[3 * b] - X[3 * a], X[3 * b + 1] - X[3 * a + 1], X[3 * b + 2] - X[3 * a + 2]};
    double len = sqrt(dot3(d, d));
    double l0 = rest_edge[j];
    double strain = len / l0 - 1.0;
    if (law == 0) {
      es += 0.5 * ks * strain * strain * l0;
      for (int k = 0; k < 3; k++) {
        double gk = ks * strain * d[k] / len;
        G[3 * b + k] += gk;
        G[3 * a + k] -= gk;
      }
    }
    /* dihedral term: 1 - cos th = 1 - n1.n2/(|n1||n2|) */
    double n1[3], n2[3];
    tri_normal(X, tri, etri[2 * j], n1);
    tri_normal(X, tri, etri[2 * j + 1], n2);
    double l1 = sqrt(dot3(n1, n1)), l2 = sqrt(dot3(n2, n2));
    double c = dot3(n1, n2) / (l1 * l2);
    eb += kb * (1.0 - c);
    /* dc/dn1 = n2/(l1 l2) - c n1/l1^2 ; dE/dn = -kb dc/dn */
    double d1[3], d2[3];
    for (int k = 0; k < 3; k++) {
      d1[k] = -kb * (n2[k] / (l1 * l2) - c * n1[k] / (l1 * l1));
      d2[k] = -kb * (n1[k] / (l1 * l2) - c * n2[k] / (l2 * l2));
    }
    add_normal_grad(X, tri, etri[2 * j], d1, G);
    add_normal_grad(X, tri, etri[2 * j + 1], d2, G);
  }
  if (law != 0) {
    /* rest length of the edge opposite each triangle vertex */
    double* ta = (double*)malloc(sizeof(double) * 3 * (size_t)ntri);
    for (int j = 0; j < ne; j++)
      for (int side = 0; side < 2; side++) {
        const int t = etri[2 * j + side];
        for (int k = 0; k < 3; k++)
          if (tri[3 * t + k] != edge[2 * j] && tri[3 * t + k] != edge[2 * j + 1]) ta[3 * t + k] = rest_edge[j];
      }
    const double h = 1e-20;
    for (int t = 0; t < ntri; t++) {
      double complex p[3][3];
      const double complex* P[3] = {p[0], p[1], p[2]};
      for (int k = 0; k < 3; k++)
        for (int d = 0; d < 3; d++) p[k][d] = X[3 * tri[3 * t + k] + d];
      es += creal(tri_law_energy(law, ks, P, ta + 3 * t));
      for (int k = 0; k < 3; k++)
        for (int d = 0; d < 3; d++) {
          const double complex keep = p[k][d];
          p[k][d] = keep + h * _Complex_I;
          G[3 * tri[3 * t + k] + d] += cimag(tri_law_energy(law, ks, P, ta + 3 * t)) / h;
          p[k][d] = keep;
        }
    }
    free(ta);
  }
  for (int k = 0; k < 3 * n; k++) F[k] = -G[k];
  free(G);
  free(edge);
  free(etri);
  if (E_s) *E_s = es;
  if (E_b) *E_b = eb;
  return 0;
}

/* ------------------------------------------------------------------ */
/* simulation object                                                   */
/* ------------------------------------------------------------------ */
orc_sim* orc_create(const orc_params* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  if (p->tau <= 0.5 || p->tau_phi <= 0.5 || p->tau_psi <= 0.5 || p->alpha <= 0.0) return NULL;
  if (p->force_form < 0 || p->force_form > 1 || (p->force_form == 1 && p->lattice != 0)) return NULL;
  for (int a = 0; a < 3; a++)
    if (!isfinite(p->fext[a])) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->p = *p;
  if (lat_make(p->lattice, &s->L)) { free(s); return NULL; }
  s->D = s->L.D;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nz = (s->D == 3) ? p->nz : 1;
  if (s->D == 2 && p->nz != 1) { free(s); return NULL; }
  s->N = (long)s->nx * s->ny * s->nz;
  const size_t N = (size_t)s->N, Q = (size_t)s->L.Q;
  for (int k = 0; k < 3; k++) {
    s->pop[k] = (double*)calloc(Q * N, sizeof(double));
    s->nxt[k] = (double*)calloc(Q * N, sizeof(double));
    s->mu[k] = (double*)calloc(N, sizeof(double));
    s->lap[k] = (double*)calloc(N, sizeof(double));
  }
  s->rho = (double*)calloc(N, sizeof(double));
  s->u = (double*)calloc(3 * N, sizeof(double));
  s->phi = (double*)calloc(N, sizeof(double));
  s->psi = (double*)calloc(N, sizeof(double));
  s->I = (double*)calloc(N, sizeof(double));
  s->grad = (double*)calloc(3 * N, sizeof(double));
  s->force = (double*)calloc(3 * N, sizeof(double));
  s->fib = (double*)calloc(3 * N, sizeof(double));
  s->sd = (double*)calloc(N, sizeof(double));
  s->seg = (int*)calloc(N, sizeof(int));
  s->bary = (double*)calloc(3 * N, sizeof(double));
  s->foot = (double*)calloc(3 * N, sizeof(double));
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  for (int k = 0; k < 3; k++) {
    free(s->pop[k]);
    free(s->nxt[k]);
    free(s->mu[k]);
    free(s->lap[k]);
  }
  free(s->rho); free(s->u); free(s->phi); free(s->psi); free(s->I); free(s->grad);
  free(s->force); free(s->fib); free(s->sd); free(s->seg); free(s->bary); free(s->foot);
  for (int m = 0; m < s->nmem; m++) {
    mem_t* M = &s->mem[m];
    free(M->X); free(M->U); free(M->F); free(M->rest); free(M->tri); free(M->edge); free(M->etri);
  }
  free(s);
}

int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

long orc_steps_done(const orc_sim* s) { return s->steps; }

int orc_add_membrane(orc_sim* s, int n, const double* X, int ntri, const int* tri, double ks,
                     double kb) {
  if (!s || !X || s->nmem >= MAXMEM) return -1;
  const int D = s->D;
  if (D == 2 && (n < 3 || ntri != 0)) return -1;
  if (D == 3 && (n < 4 || ntri < 4 || !tri)) return -1;
  mem_t* M = &s->mem[s->nmem];
  memset(M, 0, sizeof *M);
  M->n = n;
  M->ks = ks;
  M->kb = kb;
  M->X = (double*)calloc((size_t)3 * n, sizeof(double));
  M->U = (double*)calloc((size_t)3 * n, sizeof(double));
  M->F = (double*)calloc((size_t)3 * n, sizeof(double));
  for (int l = 0; l < n; l++)
    for (int a = 0; a < D; a++) M->X[3 * l + a] = X[(size_t)l * D + a];
  if (D == 2) {
    M->nedge = n;
    M->rest = (double*)malloc(sizeof(double) * n);
    /* READING: the rest length of each segment is its initial length, so the
       initial configuration carries no strain energy */
    for (int l = 0; l < n; l++) {
      int m = (l + 1) % n;
      M->rest[l] = hypot(M->X[3 * m] - M->X[3 * l], M->X[3 * m + 1] - M->X[3 * l + 1]);
    }
  } else {
    M->ntri = ntri;
    M->tri = (int*)malloc(sizeof(int) * 3 * (size_t)ntri);
    memcpy(M->tri, tri, sizeof(int) * 3 * (size_t)ntri);
    int ne = mesh_edges(n, ntri, tri, &M->edge, &M->etri);
    if (ne < 0) {
      free(M->X); free(M->U); free(M->F); free(M->tri);
      return -2;
    }
    M->nedge = ne;
    M->rest = (double*)malloc(sizeof(double) * ne);
    for (int j = 0; j < ne; j++) {
      const double *pa = M->X + 3 * M->edge[2 * j], *pb = M->X + 3 * M->edge[2 * j + 1];
      double d[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
      M->rest[j] = sqrt(dot3(d, d));
    }
  }
  return s->nmem++;
}

/* ------------------------------------------------------------------ */
/* coupling profile I, eq. Iprofile, and coupling force, eq. DiscreteCF */
/* READING: d(x, X) is the signed distance from node x to the membrane */
/* polygon (2D) or triangle mesh (3D), positive inside (the enclosed   */
/* fluid 3).  The force on a marker follows -dE_c/dX_l: the derivative */
/* of d moves the closest point, split over the closest element's      */
/* vertices with its barycentric weights.  Several membranes add their */
/* profiles.  With a band (r_cut > 0) I is exactly 0 or 1 beyond r_cut */
/* from the membrane; without one it follows eq. Iprofile everywhere.  */
/* ------------------------------------------------------------------ */

/* closest point on segment AB to P: returns squared distance, t in [0,1] */
static double seg_closest(const double* P, const double* A, const double* B, double* t_out) {
  double ex = B[0] - A[0], ey = B[1] - A[1];
  double px = P[0] - A[0], py = P[1] - A[1];
  double ee = ex * ex + ey * ey;
  double t = ee > 0.0 ? (px * ex + py * ey) / ee : 0.0;
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  double dx = px - t * ex, dy = py - t * ey;
  *t_out = t;
  return dx * dx + dy * dy;
}

/* closest point on triangle (a,b,c) to p by Voronoi-region classification;
   returns squared distance and the barycentric weights of the closest point */
static double tri_closest(const double* p, const double* a, const double* b, const double* c,
                          double* w) {
  double ab[3], ac[3], ap[3];
  for (int k = 0; k < 3; k++) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ap[k] = p[k] - a[k]; }
  double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  double u = 0, v = 0;
  if (d1 <= 0 && d2 <= 0) { u = 0; v = 0; goto done; }
  double bp[3];
  for (int k = 0; k < 3; k++) bp[k] = p[k] - b[k];
  double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3 >= 0 && d4 <= d3) { u = 1; v = 0; goto done; }
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) { u = d1 / (d1 - d3); v = 0; goto done; }
  double cp[3];
  for (int k = 0; k < 3; k++) cp[k] = p[k] - c[k];
  double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0 && d5 <= d6) { u = 0; v = 1; goto done; }
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) { u = 0; v = d2 / (d2 - d6); goto done; }
  double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    u = 1 - t; v = t; goto done;
  }
  {
    double den = 1.0 / (va + vb + vc);
    u = vb * den; v = vc * den;
  }
done:
  w[0] = 1.0 - u - v; w[1] = u; w[2] = v;
  double q[3], dd = 0;
  for (int k = 0; k < 3; k++) { q[k] = a[k] + u * ab[k] + v * ac[k] - p[k]; dd += q[k] * q[k]; }
  return dd;
}

/* even-odd crossing rule for the point-in-polygon test, half-open edges */
static int ring_inside(int n, const double* X, const double* P) {
  int in = 0;
  for (int l = 0; l < n; l++) {
    const double* A = X + 3 * l;
    const double* B = X + 3 * ((l + 1) % n);
    if ((A[1] > P[1]) != (B[1] > P[1])) {
      double xc = A[0] + (P[1] - A[1]) * (B[0] - A[0]) / (B[1] - A[1]);
      if (P[0] < xc) in = !in;
    }
  }
  return in;
}

/* even-odd rule in 3D: parity of crossings of the ray P + s e_x, s > 0, with
   the triangles (a crossing counts when the ray's (y,z) point lies in the
   triangle's (y,z) projection under a half-open rule) */
static int mesh_inside(int ntri, const int* tri, const double* X, const double* P) {
  int in = 0;
  for (int t = 0; t < ntri; t++) {
    const double *a = X + 3 * tri[3 * t], *b = X + 3 * tri[3 * t + 1], *c = X + 3 * tri[3 * t + 2];
    /* 2D edge functions in the (y,z) plane */
    double py = P[1], pz = P[2];
    double e0 = (b[1] - a[1]) * (pz - a[2]) - (b[2] - a[2]) * (py - a[1]);
    double e1 = (c[1] - b[1]) * (pz - b[2]) - (c[2] - b[2]) * (py - b[1]);
    double e2 = (a[1] - c[1]) * (pz - c[2]) - (a[2] - c[2]) * (py - c[1]);
    int pos = (e0 > 0) && (e1 > 0) && (e2 > 0);
    int neg = (e0 < 0) && (e1 < 0) && (e2 < 0);
    if (!pos && !neg) continue;
    double den = e0 + e1 + e2;
    /* barycentric weights of the projected point: a <- e1, b <- e2, c <- e0 */
    double xs = (e1 * a[0] + e2 * b[0] + e0 * c[0]) / den;
    if (xs > P[0]) in = !in;
  }
  return in;
}

/* image of lattice coordinate v nearest to centre c under period n */
static inline double near_image(double v, double c, int n, int periodic) {
  if (!periodic) return v;
  return v + n * floor((c - v) / n + 0.5);
}

/* distance from a membrane's bounding box within which nodes are searched:
   the band r_cut, or without a band 40 alpha, where (1 + tanh(d/2 alpha))/2
   already rounds to exactly 0 or 1 in FP64 (tanh(x) is 1.0 for x > 19.1) */
static double search_reach(const orc_sim* s) {
  return s->p.r_cut > 0.0 ? s->p.r_cut : 40.0 * s->p.alpha;
}

/* geometry of node n relative to membrane M: minimum-image position P and
   whether it lies in the membrane's bounding box grown by the search reach + 1 */
static int node_position(const orc_sim* s, long n, const double* lo, const double* hi,
                         const double* cen, double* P) {
  const int D = s->D;
  const double rc = search_reach(s);
  const int per[3] = {1, !s->p.wall_y, !s->p.wall_z};
  const int dims[3] = {s->nx, s->ny, s->nz};
  long r = n;
  int c[3];
  c[0] = (int)(r % s->nx); r /= s->nx;
  c[1] = (int)(r % s->ny); r /= s->ny;
  c[2] = (int)r;
  int inbox = 1;
  P[0] = P[1] = P[2] = 0.0;
  for (int a = 0; a < D; a++) {
    P[a] = near_image((double)c[a], cen[a], dims[a], per[a]);
    if (P[a] < lo[a] - rc - 1.0 || P[a] > hi[a] + rc + 1.0) inbox = 0;
  }
  return inbox;
}

static void membrane_box(const orc_sim* s, const mem_t* M, double* lo, double* hi, double* cen) {
  for (int a = 0; a < 3; a++) { lo[a] = 1e300; hi[a] = -1e300; cen[a] = 0.0; }
  for (int l = 0; l < M->n; l++)
    for (int a = 0; a < s->D; a++) {
      if (M->X[3 * l + a] < lo[a]) lo[a] = M->X[3 * l + a];
      if (M->X[3 * l + a] > hi[a]) hi[a] = M->X[3 * l + a];
    }
  for (int a = 0; a < s->D; a++) cen[a] = 0.5 * (lo[a] + hi[a]);
}

/* brute-force closest element of membrane M to P: squared distance, element
   index (lowest index on ties) and barycentric weights of the closest point */
static double closest_element(const orc_sim* s, const mem_t* M, const double* P, int* elem,
                              double* bw) {
  double best = 1e300;
  *elem = -1;
  if (s->D == 2) {
    for (int l = 0; l < M->n; l++) {
      double t;
      double d2 = seg_closest(P, M->X + 3 * l, M->X + 3 * ((l + 1) % M->n), &t);
      if (d2 < best) { best = d2; *elem = l; bw[0] = 1.0 - t; bw[1] = t; bw[2] = 0.0; }
    }
  } else {
    for (int t = 0; t < M->ntri; t++) {
      double w[3];
      double d2 = tri_closest(P, M->X + 3 * M->tri[3 * t], M->X + 3 * M->tri[3 * t + 1],
                              M->X + 3 * M->tri[3 * t + 2], w);
      if (d2 < best) { best = d2; *elem = t; bw[0] = w[0]; bw[1] = w[1]; bw[2] = w[2]; }
    }
  }
  return best;
}

static int node_inside(const orc_sim* s, const mem_t* M, const double* P) {
  if (s->D == 2) return ring_inside(M->n, M->X, P);
  /* a tiny fixed offset of the ray keeps it off mesh edges and vertices */
  double Q[3] = {P[0], P[1] + 1.2345678e-7, P[2] + 2.3456789e-7};
  return mesh_inside(M->ntri, M->tri, M->X, Q);
}

static int elem_vertex(const mem_t* M, int D, int elem, int k) {
  return (D == 2) ? (k == 0 ? elem : (elem + 1) % M->n) : M->tri[3 * elem + k];
}

static void coupling_profile(orc_sim* s, const double* psi, double* I, double* Fc_all, double* E_c,
                             int want_force) {
  const int D = s->D;
  /* rc: the band, or no band at all (beyond the search reach the profile
     is exactly 0 or 1 and its derivative below FP64 resolution) */
  const double rc = s->p.r_cut > 0.0 ? s->p.r_cut : INFINITY, al = s->p.alpha;
  const long N = s->N;
  memset(I, 0, sizeof(double) * (size_t)N);
  /* pass 1: I = sum over membranes of (1 + tanh(d/2 alpha))/2 */
  for (int m = 0; m < s->nmem; m++) {
    const mem_t* M = &s->mem[m];
    double lo[3], hi[3], cen[3];
    membrane_box(s, M, lo, hi, cen);
#pragma omp parallel for schedule(dynamic, 64)
    for (long n = 0; n < N; n++) {
      double P[3], bw[3];
      int elem;
      if (!node_position(s, n, lo, hi, cen, P)) continue; /* far outside: adds 0 */
      double d = sqrt(closest_element(s, M, P, &elem, bw));
      int inside = node_inside(s, M, P);
      if (d > rc)
        I[n] += inside ? 1.0 : 0.0;
      else
        I[n] += 0.5 * (1.0 + tanh((inside ? d : -d) / (2.0 * al)));
    }
  }
  if (E_c) {
    double e = 0.0;
    for (long n = 0; n < N; n++) {
      double dd = psi[n] - I[n];
      e += 0.5 * s->p.kappa_c * dd * dd;
    }
    *E_c = e;
  }
  if (!want_force) return;
  /* pass 2: F_v = kappa_c/(4 alpha) sum_x (psi - I) sech^2(d/2 alpha) dd/dX_v,
     dd/dX_v = -sign(d) nhat w_v with nhat the unit vector from the closest
     point to the node and w_v the closest point's barycentric weight */
  size_t off = 0;
  for (int m = 0; m < s->nmem; m++) {
    const mem_t* M = &s->mem[m];
    double* Fc = Fc_all + off;
    memset(Fc, 0, sizeof(double) * 3 * (size_t)M->n);
    double lo[3], hi[3], cen[3];
    membrane_box(s, M, lo, hi, cen);
#pragma omp parallel for schedule(dynamic, 64)
    for (long n = 0; n < N; n++) {
      double P[3], bw[3];
      int elem;
      s->seg[n] = -1;
      if (!node_position(s, n, lo, hi, cen, P)) continue;
      double d = sqrt(closest_element(s, M, P, &elem, bw));
      if (d > rc || d == 0.0) continue;
      int inside = node_inside(s, M, P);
      double foot[3] = {0, 0, 0};
      int nv = (D == 2) ? 2 : 3;
      for (int k = 0; k < nv; k++)
        for (int a = 0; a < D; a++) foot[a] += bw[k] * M->X[3 * elem_vertex(M, D, elem, k) + a];
      s->seg[n] = elem;
      s->sd[n] = inside ? d : -d;
      for (int a = 0; a < 3; a++) {
        s->bary[3 * n + a] = bw[a];
        s->foot[3 * n + a] = (P[a] - foot[a]) / d;
      }
    }
    /* serial accumulation in node order */
    for (long n = 0; n < N; n++) {
      int elem = s->seg[n];
      if (elem < 0) continue;
      double sd = s->sd[n], sg = sd > 0.0 ? 1.0 : -1.0;
      double ch = cosh(sd / (2.0 * al));
      double wgt = s->p.kappa_c / (4.0 * al) * (psi[n] - I[n]) / (ch * ch);
      int nv = (D == 2) ? 2 : 3;
      for (int k = 0; k < nv; k++) {
        int v = elem_vertex(M, D, elem, k);
        for (int a = 0; a < D; a++) Fc[3 * v + a] += wgt * (-sg * s->foot[3 * n + a] * s->bary[3 * n + k]);
      }
    }
    off += 3 * (size_t)M->n;
  }
}

int orc_coupling(orc_sim* s, const double* psi, double* I, double* Fc, double* E_c) {
  coupling_profile(s, psi, I, Fc, E_c, Fc != NULL);
  return 0;
}

/* ------------------------------------------------------------------ */
/* the time step                                                       */
/* ------------------------------------------------------------------ */
static void compute_moments(orc_sim* s, double* const* pop, double* rho, double* u, double* phi,
                            double* psi) {
  const lat_t* L = &s->L;
  const long N = s->N;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double r = 0, m[3] = {0, 0, 0}, ph = 0, ps = 0;
    for (int i = 0; i < L->Q; i++) {
      double fi = pop[0][(size_t)i * N + n];
      r += fi;
      for (int a = 0; a < 3; a++) m[a] += L->c[i][a] * fi;
      ph += pop[1][(size_t)i * N + n];
      ps += pop[2][(size_t)i * N + n];
    }
    rho[n] = r;
    for (int a = 0; a < 3; a++) u[3 * n + a] = m[a] / r;
    phi[n] = ph;
    psi[n] = ps;
  }
}

/* chemical potentials on the whole lattice from rho, phi, psi and I */
/* ------------------------------------------------------------------ */
/* pressure tensor, Appendix A.  The gradient part uses the kappa mixing  */
/* matrix printed there (the Hessian of the gradient energy in rho, phi,  */
/* psi).  READING: the bulk part is taken from its definition,            */
/* p_b' = sum_q q mu_q^b - f_b = sum_m [C_m f_m'(C_m) - f_m(C_m)] with    */
/* f_m = kappa_m/2 C_m^2 (1 - C_m)^2, not from the printed polynomial,    */
/* which differs from it by a non-constant term; the ideal gas rho c_s^2  */
/* is left out as in the potential form (it cancels in eq. ForceFE).      */
/* ------------------------------------------------------------------ */
int orc_pressure_tensor(const orc_params* p, int D, const double* q, const double* g, const double* l,
                        double* P) {
  if (!p || D < 2 || D > 3) return -1;
  const double k1 = p->kappa1, k2 = p->kappa2, k3 = p->kappa3, a2 = p->alpha * p->alpha;
  double K[3][3] = {{(k1 + k2) / 4.0, (k1 - k2) / 4.0, -(k1 + k2) / 4.0},
                    {(k1 - k2) / 4.0, (k1 + k2) / 4.0, -(k1 - k2) / 4.0},
                    {-(k1 + k2) / 4.0, -(k1 - k2) / 4.0, (k1 + k2 + 4.0 * k3) / 4.0}};
  double C[3];
  orc_concentrations(p, q[0], q[1], q[2], C);
  const double km[3] = {k1, k2, k3};
  if (!equal_densities(p)) {
    /* the gradient energy's Hessian in (rho, phi, psi): A^T diag(kappa) A */
    double A[3][3];
    conc_matrix(p, A);
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        K[i][j] = 0.0;
        for (int m = 0; m < 3; m++) K[i][j] += A[m][i] * km[m] * A[m][j];
      }
  }
  double pb = 0.0;
  for (int m = 0; m < 3; m++) {
    const double c = C[m];
    const double f = 0.5 * km[m] * c * c * (1.0 - c) * (1.0 - c);
    const double fp = km[m] * c * (1.0 - c) * (1.0 - 2.0 * c);
    pb += c * fp - f;
  }
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) P[3 * a + b] = (a == b && a < D) ? pb : 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double gg = 0.0;
      for (int a = 0; a < D; a++) gg += g[3 * i + a] * g[3 * j + a];
      for (int a = 0; a < D; a++)
        for (int b = 0; b < D; b++) {
          double t = g[3 * i + a] * g[3 * j + b];
          if (a == b) t -= 0.5 * gg + q[i] * l[j];
          P[3 * a + b] += a2 * K[i][j] * t;
        }
    }
  return 0;
}

/* p' at lattice point (x, y) of the mirror-extended fields: a point beyond
   a wall takes the values of its mirror node, with the gradient's component
   normal to the wall reversed (the fields are even about the wall) */
static void pressure_at(const orc_sim* s, const double* const qf[3], const double* const gf[3],
                        const double* const lf[3], int x, int y, double* P) {
  const int xx = wrapi(x, s->nx);
  int yy = y, flip = 0;
  if (s->p.wall_y) {
    if (y < 0) { yy = -1 - y; flip = 1; }
    if (y >= s->ny) { yy = 2 * s->ny - 1 - y; flip = 1; }
  } else {
    yy = wrapi(y, s->ny);
  }
  const long n = nid(s, xx, yy, 0);
  double q[3], g[9] = {0}, l[3];
  for (int k = 0; k < 3; k++) {
    q[k] = qf[k][n];
    l[k] = lf[k][n];
    g[3 * k] = gf[k][2 * n];
    g[3 * k + 1] = flip ? -gf[k][2 * n + 1] : gf[k][2 * n + 1];
  }
  orc_pressure_tensor(&s->p, 2, q, g, l, P);
}

/* -div p' (eq. ForceFE, divergence form) by the isotropic gradient stencil
   applied to the tensor's columns, 2 components per node into F2 */
static void div_pressure(const orc_sim* s, double* F2) {
  const long N = s->N;
  double* g[3];
  for (int k = 0; k < 3; k++) g[k] = (double*)malloc(sizeof(double) * 2 * (size_t)N);
  orc_grad_lap(s, s->rho, g[0], s->lap[0]);
  orc_grad_lap(s, s->phi, g[1], s->lap[1]);
  orc_grad_lap(s, s->psi, g[2], s->lap[2]);
  const double* const qf[3] = {s->rho, s->phi, s->psi};
  const double* const gf[3] = {g[0], g[1], g[2]};
  const double* const lf[3] = {s->lap[0], s->lap[1], s->lap[2]};
  const lat_t* L = &s->L;
#pragma omp parallel for collapse(2) schedule(static)
  for (int y = 0; y < s->ny; y++)
    for (int x = 0; x < s->nx; x++) {
      double d[2] = {0.0, 0.0};
      for (int i = 0; i < L->Q; i++) {
        double P[9];
        pressure_at(s, qf, gf, lf, x + L->c[i][0], y + L->c[i][1], P);
        for (int a = 0; a < 2; a++)
          for (int b = 0; b < 2; b++) d[a] += L->w[i] * L->c[i][b] * P[3 * a + b];
      }
      const long n = nid(s, x, y, 0);
      F2[2 * n] = -d[0] / CS2;
      F2[2 * n + 1] = -d[1] / CS2;
    }
  for (int k = 0; k < 3; k++) free(g[k]);
}

static void compute_mu(orc_sim* s) {
  orc_grad_lap(s, s->rho, NULL, s->lap[0]);
  orc_grad_lap(s, s->phi, NULL, s->lap[1]);
  orc_grad_lap(s, s->psi, NULL, s->lap[2]);
  const long N = s->N;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double m3[3];
    orc_mu(&s->p, s->rho[n], s->phi[n], s->psi[n], s->lap[0][n], s->lap[1][n], s->lap[2][n],
           s->I[n], m3);
    s->mu[0][n] = m3[0];
    s->mu[1][n] = m3[1];
    s->mu[2][n] = m3[2];
  }
}

int orc_set_fields(orc_sim* s, const double* rho, const double* phi, const double* psi,
                   const double* ux, const double* uy, const double* uz) {
  if (!s || !rho || !phi || !psi) return -1;
  const long N = s->N;
  for (long n = 0; n < N; n++) {
    if (!(rho[n] > 0.0)) return -2;
    s->rho[n] = rho[n];
    s->phi[n] = phi[n];
    s->psi[n] = psi[n];
    s->u[3 * n + 0] = ux ? ux[n] : 0.0;
    s->u[3 * n + 1] = uy ? uy[n] : 0.0;
    s->u[3 * n + 2] = (uz && s->D == 3) ? uz[n] : 0.0;
  }
  coupling_profile(s, s->psi, s->I, NULL, NULL, 0);
  compute_mu(s);
  const lat_t* L = &s->L;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; n++) {
    double e[MAXQ], sh[MAXQ];
    feq_all(L, s->rho[n], s->u + 3 * n, e);
    feq_pressure_shift(L, &s->p, s->phi[n], s->psi[n], sh);
    for (int i = 0; i < L->Q; i++) s->pop[0][(size_t)i * N + n] = e[i] + sh[i];
    geq_all(L, s->phi[n], s->mu[1][n], s->p.gamma_phi, s->u + 3 * n, e);
    for (int i = 0; i < L->Q; i++) s->pop[1][(size_t)i * N + n] = e[i];
    geq_all(L, s->psi[n], s->mu[2][n], s->p.gamma_psi, s->u + 3 * n, e);
    for (int i = 0; i < L->Q; i++) s->pop[2][(size_t)i * N + n] = e[i];
  }
  memset(s->force, 0, sizeof(double) * 3 * (size_t)N);
  s->steps = 0;
  s->ready = 1;
  return 0;
}

static size_t total_markers(const orc_sim* s) {
  size_t t = 0;
  for (int m = 0; m < s->nmem; m++) t += (size_t)s->mem[m].n;
  return t;
}

/* BGK collision of the three population sets at one node, eq. LBE:
   f uses the exact-difference forcing f^eq(rho, u + du) - f^eq(rho, u) with
   du = F/rho (eq. VelCorrection); g and h relax to equilibria taken at the
   actual velocity v = u + du/2 (eq. ActualFluidVel). */
static void collide_node(const lat_t* L, const orc_params* p, double in[3][MAXQ], double rho,
                         const double* u, double phi, double psi, double mu_phi, double mu_psi,
                         const double* F, double post[3][MAXQ]) {
  double du[3], up[3], v[3];
  for (int a = 0; a < 3; a++) {
    du[a] = F[a] / rho;
    up[a] = u[a] + du[a];
    v[a] = u[a] + 0.5 * du[a];
  }
  double fe[MAXQ], fe2[MAXQ], ge[MAXQ], he[MAXQ], sh[MAXQ];
  feq_all(L, rho, u, fe);
  feq_all(L, rho, up, fe2);
  geq_all(L, phi, mu_phi, p->gamma_phi, v, ge);
  geq_all(L, psi, mu_psi, p->gamma_psi, v, he);
  feq_pressure_shift(L, p, phi, psi, sh);
  for (int i = 0; i < L->Q; i++) {
    /* the pressure shift moves the BGK target only: it cancels in the
       exact-difference term */
    post[0][i] = in[0][i] - (in[0][i] - (fe[i] + sh[i])) / p->tau + (fe2[i] - fe[i]);
    post[1][i] = in[1][i] - (in[1][i] - ge[i]) / p->tau_phi;
    post[2][i] = in[2][i] - (in[2][i] - he[i]) / p->tau_psi;
  }
}

int orc_collide(const orc_params* p, const double* in, const double* F, double mu_phi,
                double mu_psi, double* out) {
  lat_t L;
  if (lat_make(p->lattice, &L)) return -1;
  double pin[3][MAXQ], post[3][MAXQ];
  double rho = 0, m[3] = {0, 0, 0}, phi = 0, psi = 0;
  for (int i = 0; i < L.Q; i++) {
    for (int k = 0; k < 3; k++) pin[k][i] = in[k * L.Q + i];
    rho += pin[0][i];
    for (int a = 0; a < 3; a++) m[a] += L.c[i][a] * pin[0][i];
    phi += pin[1][i];
    psi += pin[2][i];
  }
  double u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
  double FF[3] = {F[0], F[1], L.D == 3 ? F[2] : 0.0};
  collide_node(&L, p, pin, rho, u, phi, psi, mu_phi, mu_psi, FF, post);
  for (int i = 0; i < L.Q; i++)
    for (int k = 0; k < 3; k++) out[k * L.Q + i] = post[k][i];
  return 0;
}

/* one step t -> t+1, in the order of Sec. 3.3:
   moments(t); I(X(t)); mu(t); F_mem(X(t)); spread; force; collide+stream;
   interpolate v at t+1 at the markers; X(t+1) = X(t) + U. */
static void one_step(orc_sim* s) {
  const lat_t* L = &s->L;
  const long N = s->N;
  const int D = s->D;
  const size_t Q = (size_t)L->Q;

  /* 1. moments, eq. MomentsDFs */
  compute_moments(s, s->pop, s->rho, s->u, s->phi, s->psi);

  /* 2-3. coupling profile and coupling forces, then chemical potentials */
  size_t nm = total_markers(s);
  double* Fc = (double*)calloc(3 * (nm ? nm : 1), sizeof(double));
  coupling_profile(s, s->psi, s->I, Fc, NULL, 1);
  compute_mu(s);

  /* 4. membrane forces (eq. DiscreteTF) and spreading (eq. Spreading) */
  memset(s->fib, 0, sizeof(double) * 3 * (size_t)N);
  size_t off = 0;
  for (int m = 0; m < s->nmem; m++) {
    mem_t* M = &s->mem[m];
    double* Fm = (double*)calloc(3 * (size_t)M->n, sizeof(double));
    if (D == 2) {
      double* X2 = (double*)malloc(sizeof(double) * 2 * M->n);
      double* F2 = (double*)malloc(sizeof(double) * 2 * M->n);
      for (int l = 0; l < M->n; l++) { X2[2 * l] = M->X[3 * l]; X2[2 * l + 1] = M->X[3 * l + 1]; }
      orc_ring_forces_law(M->n, X2, M->rest, M->ks, M->kb, M->law, F2, NULL, NULL);
      for (int l = 0; l < M->n; l++) { Fm[3 * l] = F2[2 * l]; Fm[3 * l + 1] = F2[2 * l + 1]; }
      free(X2);
      free(F2);
    } else {
      orc_mesh_forces_law(M->n, M->X, M->ntri, M->tri, M->rest, M->ks, M->kb, M->law, Fm, NULL, NULL);
    }
    for (int l = 0; l < M->n; l++)
      for (int a = 0; a < 3; a++) {
        M->F[3 * l + a] = Fm[3 * l + a] + Fc[off + 3 * (size_t)l + a];
      }
    free(Fm);
    off += 3 * (size_t)M->n;
  }
  free(Fc);
  for (int m = 0; m < s->nmem; m++) {
    mem_t* M = &s->mem[m];
    for (int l = 0; l < M->n; l++) {
      spread_ctx k = {s->fib, M->F + 3 * (size_t)l, 3};
      stencil_visit(s, M->X + 3 * (size_t)l, spread_cb, &k);
    }
  }

  /* 5. force f = f_FE + f_IB + f_ext (eq. ForcingTermLBE), with
        f_FE = -rho grad mu_rho - phi grad mu_phi - psi grad mu_psi'
        (potential form) or -div p' - psi grad kappa_c (psi - I)
        (divergence form) */
  if (s->p.force_form == 1) {
    double* F2 = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    double* cp = (double*)malloc(sizeof(double) * (size_t)N);
    double* gc = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    div_pressure(s, F2);
    for (long n = 0; n < N; n++) cp[n] = s->p.kappa_c * (s->psi[n] - s->I[n]);
    orc_grad_lap(s, cp, gc, NULL);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
      for (int a = 0; a < 3; a++) s->force[3 * n + a] = 0.0;
      for (int a = 0; a < 2; a++)
        s->force[3 * n + a] = F2[2 * n + a] - s->psi[n] * gc[2 * n + a] + s->fib[3 * n + a] + s->p.fext[a];
    }
    free(F2);
    free(cp);
    free(gc);
  } else {
    double* g0 = (double*)malloc(sizeof(double) * D * (size_t)N);
    double* g1 = (double*)malloc(sizeof(double) * D * (size_t)N);
    double* g2 = (double*)malloc(sizeof(double) * D * (size_t)N);
    orc_grad_lap(s, s->mu[0], g0, NULL);
    orc_grad_lap(s, s->mu[1], g1, NULL);
    orc_grad_lap(s, s->mu[2], g2, NULL);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) {
      for (int a = 0; a < 3; a++) s->force[3 * n + a] = 0.0;
      for (int a = 0; a < D; a++)
        s->force[3 * n + a] = -s->rho[n] * g0[n * D + a] - s->phi[n] * g1[n * D + a] -
                              s->psi[n] * g2[n * D + a] + s->fib[3 * n + a] + s->p.fext[a];
    }
    free(g0);
    free(g1);
    free(g2);
  }

  /* 6. collide (eq. LBE with the exact-difference forcing for f) and stream */
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < s->nz; z++)
    for (int y = 0; y < s->ny; y++)
      for (int x = 0; x < s->nx; x++) {
        long n = nid(s, x, y, z);
        double in[3][MAXQ], post[3][MAXQ];
        for (size_t i = 0; i < Q; i++)
          for (int k = 0; k < 3; k++) in[k][i] = s->pop[k][i * N + n];
        collide_node(L, &s->p, in, s->rho[n], s->u + 3 * n, s->phi[n], s->psi[n],
                     s->mu[1][n], s->mu[2][n], s->force + 3 * n, post);
        for (size_t i = 0; i < Q; i++) {
          long dn = stream_dest(s, x, y, z, (int)i);
          for (int k = 0; k < 3; k++) {
            if (dn >= 0)
              s->nxt[k][i * N + dn] = post[k][i];
            else /* half-way bounce-back: returns to this node reversed */
              s->nxt[k][(size_t)L->opp[i] * N + n] = post[k][i];
          }
        }
      }
  for (int k = 0; k < 3; k++) {
    double* t = s->pop[k];
    s->pop[k] = s->nxt[k];
    s->nxt[k] = t;
  }

  /* 7. marker velocities: v at t+1 interpolated at X(t) (eq. Interpolation),
        then Euler update (eq. UpdatedXl).  READING: the force at t+1 needs
        X(t+1), so the half-force correction at t+1 uses the force of step t:
        v* = u(t+1) + f(t) / (2 rho(t+1)). */
  if (s->nmem > 0) {
    double* vstar = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    compute_moments(s, s->pop, s->rho, s->u, s->phi, s->psi);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++)
      for (int a = 0; a < 3; a++) vstar[3 * n + a] = s->u[3 * n + a] + 0.5 * s->force[3 * n + a] / s->rho[n];
    for (int m = 0; m < s->nmem; m++) {
      mem_t* M = &s->mem[m];
      for (int l = 0; l < M->n; l++) {
        interp_ctx k = {vstar, {0, 0, 0}, 3};
        stencil_visit(s, M->X + 3 * (size_t)l, interp_cb, &k);
        for (int a = 0; a < 3; a++) M->U[3 * l + a] = k.acc[a];
      }
      for (int l = 0; l < M->n; l++)
        for (int a = 0; a < D; a++) M->X[3 * l + a] += M->U[3 * l + a];
    }
    free(vstar);
  }
  s->steps++;
}

int orc_step(orc_sim* s, int n_steps) {
  if (!s || !s->ready || n_steps < 0) return -1;
  for (int k = 0; k < n_steps; k++) one_step(s);
  return 0;
}

int orc_fe_force(orc_sim* s, int form, double* F) {
  if (!s || !s->ready || !F || form < 0 || form > 1 || (form == 1 && s->D != 2)) return -1;
  const long N = s->N;
  const int D = s->D;
  compute_moments(s, s->pop, s->rho, s->u, s->phi, s->psi);
  for (long n = 0; n < 3 * N; n++) F[n] = 0.0;
  if (form == 1) {
    double* F2 = (double*)malloc(sizeof(double) * 2 * (size_t)N);
    div_pressure(s, F2);
    for (long n = 0; n < N; n++) {
      F[3 * n] = F2[2 * n];
      F[3 * n + 1] = F2[2 * n + 1];
    }
    free(F2);
    return 0;
  }
  /* potential form without the coupling term: mu at I = psi */
  double* mu[3];
  double* gm = (double*)malloc(sizeof(double) * D * (size_t)N);
  for (int k = 0; k < 3; k++) mu[k] = (double*)malloc(sizeof(double) * (size_t)N);
  orc_grad_lap(s, s->rho, NULL, s->lap[0]);
  orc_grad_lap(s, s->phi, NULL, s->lap[1]);
  orc_grad_lap(s, s->psi, NULL, s->lap[2]);
  for (long n = 0; n < N; n++) {
    double m3[3];
    orc_mu(&s->p, s->rho[n], s->phi[n], s->psi[n], s->lap[0][n], s->lap[1][n], s->lap[2][n], s->psi[n], m3);
    for (int k = 0; k < 3; k++) mu[k][n] = m3[k];
  }
  const double* qv[3] = {s->rho, s->phi, s->psi};
  for (int k = 0; k < 3; k++) {
    orc_grad_lap(s, mu[k], gm, NULL);
    for (long n = 0; n < N; n++)
      for (int a = 0; a < D; a++) F[3 * n + a] -= qv[k][n] * gm[(size_t)n * D + a];
  }
  for (int k = 0; k < 3; k++) free(mu[k]);
  free(gm);
  return 0;
}

int orc_get_fields(const orc_sim* s, double* rho, double* c1, double* c2, double* c3, double* ux,
                   double* uy, double* uz) {
  if (!s || !s->ready) return -1;
  const lat_t* L = &s->L;
  const long N = s->N;
  for (long n = 0; n < N; n++) {
    double r = 0, m[3] = {0, 0, 0}, ph = 0, ps = 0;
    for (int i = 0; i < L->Q; i++) {
      double fi = s->pop[0][(size_t)i * N + n];
      r += fi;
      for (int a = 0; a < 3; a++) m[a] += L->c[i][a] * fi;
      ph += s->pop[1][(size_t)i * N + n];
      ps += s->pop[2][(size_t)i * N + n];
    }
    /* eq. VariableTransform inverted (with component densities, the map of
       orc_concentrations) */
    double C[3];
    orc_concentrations(&s->p, r, ph, ps, C);
    if (rho) rho[n] = r;
    if (c1) c1[n] = C[0];
    if (c2) c2[n] = C[1];
    if (c3) c3[n] = C[2];
    if (ux) ux[n] = m[0] / r;
    if (uy) uy[n] = m[1] / r;
    if (uz) uz[n] = m[2] / r;
  }
  return 0;
}

int orc_set_membrane_law(orc_sim* s, int id, int law) {
  if (!s || id < 0 || id >= s->nmem || law < 0 || law > 2) return -1;
  s->mem[id].law = law;
  return 0;
}

int orc_set_rest(orc_sim* s, int id, const double* rest) {
  if (!s || !rest || id < 0 || id >= s->nmem) return -1;
  mem_t* M = &s->mem[id];
  for (int j = 0; j < M->nedge; j++)
    if (!(rest[j] > 0.0) || !isfinite(rest[j])) return -1;
  for (int j = 0; j < M->nedge; j++) M->rest[j] = rest[j];
  return 0;
}

int orc_get_membrane(const orc_sim* s, int id, double* X, double* U, double* F) {
  if (!s || id < 0 || id >= s->nmem) return -1;
  const mem_t* M = &s->mem[id];
  const int D = s->D;
  for (int l = 0; l < M->n; l++)
    for (int a = 0; a < D; a++) {
      if (X) X[(size_t)l * D + a] = M->X[3 * l + a];
      if (U) U[(size_t)l * D + a] = M->U[3 * l + a];
      if (F) F[(size_t)l * D + a] = M->F[3 * l + a];
    }
  return 0;
}

/* energies at the current state (eqs. Densities, LandauFE, CouplingE,
   DiscreteSE, DiscreteBE); fixed-order serial sums */
int orc_energy(orc_sim* s, orc_energies* out) {
  if (!s || !s->ready || !out) return -1;
  const long N = s->N;
  const int D = s->D;
  memset(out, 0, sizeof *out);
  compute_moments(s, s->pop, s->rho, s->u, s->phi, s->psi);
  double* C[3];
  double* G = (double*)malloc(sizeof(double) * D * (size_t)N);
  for (int m = 0; m < 3; m++) C[m] = (double*)malloc(sizeof(double) * (size_t)N);
  for (long n = 0; n < N; n++) {
    double c[3];
    orc_concentrations(&s->p, s->rho[n], s->phi[n], s->psi[n], c);
    for (int m = 0; m < 3; m++) C[m][n] = c[m];
  }
  const double kap[3] = {s->p.kappa1, s->p.kappa2, s->p.kappa3};
  const double a2 = s->p.alpha * s->p.alpha;
  for (int m = 0; m < 3; m++) {
    orc_grad_lap(s, C[m], G, NULL);
    double mass = 0, fb = 0, fg = 0;
    for (long n = 0; n < N; n++) {
      double c = C[m][n];
      mass += c;
      fb += 0.5 * kap[m] * c * c * (1.0 - c) * (1.0 - c);
      double gg = 0;
      for (int a = 0; a < D; a++) gg += G[n * D + a] * G[n * D + a];
      fg += 0.5 * a2 * kap[m] * gg;
    }
    out->mass[m] = mass;
    out->F_bulk += fb;
    out->F_grad += fg;
  }
  double ek = 0, pid = 0;
  for (long n = 0; n < N; n++) {
    double uu = 0;
    for (int a = 0; a < 3; a++) uu += s->u[3 * n + a] * s->u[3 * n + a];
    ek += 0.5 * s->rho[n] * uu;
    /* c_s^2 rho ln rho; with component densities that of n: c_s^2 Mb n ln n */
    if (equal_densities(&s->p)) {
      pid += CS2 * s->rho[n] * log(s->rho[n]);
    } else {
      double M[3];
      mw_get(&s->p, M);
      const double Mb = 0.5 * (M[0] + M[1]);
      const double nn = C[0][n] + C[1][n] + C[2][n];
      pid += CS2 * Mb * nn * log(nn);
    }
  }
  out->E_kin = ek;
  out->p_ideal = pid;
  coupling_profile(s, s->psi, s->I, NULL, &out->E_c, 0);
  for (int m = 0; m < s->nmem; m++) {
    mem_t* M = &s->mem[m];
    double es = 0, eb = 0;
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)M->n);
    if (D == 2) {
      double* X2 = (double*)malloc(sizeof(double) * 2 * M->n);
      for (int l = 0; l < M->n; l++) { X2[2 * l] = M->X[3 * l]; X2[2 * l + 1] = M->X[3 * l + 1]; }
      orc_ring_forces_law(M->n, X2, M->rest, M->ks, M->kb, M->law, F, &es, &eb);
      free(X2);
    } else {
      orc_mesh_forces_law(M->n, M->X, M->ntri, M->tri, M->rest, M->ks, M->kb, M->law, F, &es, &eb);
    }
    free(F);
    out->E_s += es;
    out->E_b += eb;
  }
  for (int m = 0; m < 3; m++) free(C[m]);
  free(G);
  return 0;
}
