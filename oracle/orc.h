/*
 * orc.h -- plain FP64 CPU oracle of the ternary free-energy lattice Boltzmann
 * + immersed-boundary time step (Pepona, Shek, Semprebon, Krueger,
 * Kusumaatmaja, "Modelling ternary fluids in contact with elastic membranes").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP library
 * against the paper.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * helper with the GPU path.
 *
 * Conventions
 *   - Lattice nodes sit at integer coordinates; node (x,y,z) has linear index
 *     x + nx*(y + ny*z).  x is always periodic; y (and z in 3D) are periodic
 *     or bounded by half-way bounce-back walls at y = -1/2 and y = ny - 1/2.
 *   - Everything is double precision.  Arrays passed in are copied; arrays
 *     passed out are filled by the callee and owned by the caller.
 *   - Every function returns 0 on success and a negative code on bad input.
 */
#ifndef ORC_H
#define ORC_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int lattice;            /* 0: D2Q9 (Sec. 3.1), 1: D3Q19                        */
  int nx, ny, nz;         /* nz = 1 for D2Q9                                      */
  int wall_y, wall_z;     /* 0 periodic, 1 half-way bounce-back walls             */
  double tau, tau_phi, tau_psi;     /* relaxation times, eq. RelaxationTimes      */
  double gamma_phi, gamma_psi;      /* mobility prefactors Gamma, eq. EDF         */
  double kappa1, kappa2, kappa3;    /* Landau parameters, eq. LandauFE            */
  double alpha;                     /* interface width, eq. LandauFE              */
  double kappa_c;                   /* membrane coupling, eq. CouplingE           */
  double r_cut;           /* coupling band: beyond this distance from a membrane
                             the profile I is exactly 0 or 1 and the node adds
                             no coupling force.  <= 0: no band, the profile of
                             eq. Iprofile everywhere (it is searched within
                             40*alpha of a membrane's box, where the FP64 tanh
                             is already exactly +-1).                          */
  int force_form;         /* free-energy force of eq. ForceFE: 0 potential form
                             -rho grad mu_rho - phi grad mu_phi - psi grad mu_psi',
                             1 divergence form -div p' - psi grad kappa_c(psi - I)
                             with the pressure tensor of Appendix A (D2Q9 only)  */
  double fext[3];         /* uniform external force density f_ext of eq.
                             ForcingTermLBE (zero in the paper's runs)           */
  double mw[3];           /* component densities M_w,m of eq. MassDensity
                             (rho = sum_m M_m C_m); <= 0 means 1.  All equal to
                             1 is the paper's model; otherwise the extension the
                             paper names in its conclusions, see orc.c          */
} orc_params;

/* energies and conserved sums, all FP64 */
typedef struct {
  double mass[3];         /* sum over nodes of C1, C2, C3                          */
  double F_bulk;          /* sum kappa_m/2 C_m^2 (1-C_m)^2                          */
  double F_grad;          /* sum alpha^2 kappa_m/2 |grad C_m|^2                     */
  double E_c;             /* kappa_c/2 sum (psi - I)^2, eq. DiscreteCE              */
  double E_s, E_b;        /* membrane strain / bending, eqs. DiscreteSE, DiscreteBE */
  double E_kin;           /* 1/2 sum rho |u|^2 (bare velocity)                      */
  double p_ideal;         /* sum c_s^2 rho ln rho                                   */
} orc_energies;

typedef struct orc_sim orc_sim;

orc_sim* orc_create(const orc_params* p);

/* Pressure tensor p' of Appendix A without the ideal-gas part, at one point
 * from the values q = (rho, phi, psi), their gradients g[q][a] and
 * Laplacians l[q]; P receives the D x D components (row-major 3 x 3).  */
int orc_pressure_tensor(const orc_params* p, int D, const double* q, const double* g, const double* l,
                        double* P);

/* Free-energy force (no coupling term, no membrane force) of the current
 * populations in the given form (0 potential, 1 divergence; D2Q9 only for
 * 1): F receives 3 values per node.  */
int orc_fe_force(orc_sim* s, int form, double* F);
void     orc_destroy(orc_sim* s);
int      orc_set_threads(int n);   /* OpenMP threads for node loops; returns the count used */

/* Membranes.  2D: closed ring of n_nodes markers (n_tris = 0, tris = NULL).
 * 3D: closed triangle mesh (n_tris triangles, tris = 3*n_tris vertex ids,
 * counter-clockwise seen from outside).  rest = NULL: rest lengths are the
 * initial edge lengths.  Returns the membrane id (>= 0) or a negative code.  */
int orc_add_membrane(orc_sim* s, int n_nodes, const double* X, int n_tris, const int* tris,
                     double kappa_s, double kappa_b);

/* Strain law of membrane id: 0 eq. DiscreteSE (2D) or edge springs (3D,
 * the default), 1 neo-Hookean, 2 Skalak; 2D rings take them at plane strain
 * with the same small-strain modulus, 3D meshes per triangle with shear
 * modulus kappa_s (Skalak C = 1).  Rest lengths of membrane id: 2D, per
 * segment l -> l+1; 3D, per edge in order of first appearance over the
 * triangles' edges (v_k, v_k+1).                                          */
int orc_set_membrane_law(orc_sim* s, int id, int law);
int orc_set_rest(orc_sim* s, int id, const double* rest);

/* Macroscopic initial fields (N each; uz may be NULL in 2D).  Builds the
 * equilibrium populations, using the membranes added so far for I.          */
int orc_set_fields(orc_sim* s, const double* rho, const double* phi, const double* psi,
                   const double* ux, const double* uy, const double* uz);

int orc_step(orc_sim* s, int n_steps);
long orc_steps_done(const orc_sim* s);

/* rho, C1, C2, C3 and the bare velocity u = sum c_i f_i / rho (any may be NULL) */
int orc_get_fields(const orc_sim* s, double* rho, double* c1, double* c2, double* c3,
                   double* ux, double* uy, double* uz);
/* markers: positions X (n*d), last interpolated velocity U, last total force F */
int orc_get_membrane(const orc_sim* s, int id, double* X, double* U, double* F);
int orc_energy(orc_sim* s, orc_energies* out);

/* ---- pieces exposed for unit pins (pure functions of their inputs) ---- */
double orc_peskin(double r);                              /* eq. DiscreteDirac   */
/* lattice tables: Q, velocities c (Q*3 ints), weights w (Q) */
int orc_lattice(int lattice, int* Q, int* c, double* w);
/* f^eq(rho,u) for all i, eq. EDF */
int orc_feq(int lattice, double rho, const double* u, double* out);
/* g^eq / h^eq for order parameter q with chemical potential mu, mobility Gamma */
int orc_geq(int lattice, double q, double mu, double Gamma, const double* v, double* out);
/* chemical potentials (mu_rho without its ideal-gas part, mu_phi, mu_psi')
   from local values and Laplacians, Appendix A (equal densities) or the
   general form through the concentrations (unequal densities) */
void orc_mu(const orc_params* p, double rho, double phi, double psi,
            double lap_rho, double lap_phi, double lap_psi, double I, double* mu3);
/* the same always through the concentration map of mw (for the pin that
   the general form reduces to Appendix A when every M_m is 1) */
void orc_mu_general(const orc_params* p, double rho, double phi, double psi,
                    double lap_rho, double lap_phi, double lap_psi, double I, double* mu3);
/* concentrations C1..C3 from rho, phi, psi under the component densities */
void orc_concentrations(const orc_params* p, double rho, double phi, double psi, double* C);
/* one BGK collision (eq. LBE) of the populations in = [f(Q), g(Q), h(Q)] of
   one node under force F, with the given chemical potentials; out likewise */
int orc_collide(const orc_params* p, const double* in, const double* F, double mu_phi,
                double mu_psi, double* out);
/* isotropic finite differences on a field q (N values) of simulation s */
int orc_grad_lap(const orc_sim* s, const double* q, double* grad /*N*d*/, double* lap /*N*/);
/* 2D ring membrane energies and forces F = -dE/dX (strain + bending) */
int orc_ring_forces(int n, const double* X, const double* rest, double kappa_s, double kappa_b,
                    double* F, double* E_s, double* E_b);
/* the same with the strain law of orc_set_membrane_law */
int orc_ring_forces_law(int n, const double* X, const double* rest, double kappa_s, double kappa_b,
                        int law, double* F, double* E_s, double* E_b);
/* 3D mesh membrane energies and forces; _law: with the strain law above */
int orc_mesh_forces_law(int n, const double* X, int n_tris, const int* tris, const double* rest_edge,
                        double kappa_s, double kappa_b, int law, double* F, double* E_s, double* E_b);
int orc_mesh_forces(int n, const double* X, int n_tris, const int* tris, const double* rest_edge,
                    double kappa_s, double kappa_b, double* F, double* E_s, double* E_b);
/* coupling field I (N) and coupling forces on the markers of every membrane,
   given psi (N); Fc has 3 doubles per marker, membranes concatenated */
int orc_coupling(orc_sim* s, const double* psi, double* I, double* Fc, double* E_c);
/* spreading of marker forces (d per marker) onto the lattice (N*d), eq. Spreading */
int orc_spread(const orc_sim* s, int n, const double* X, const double* F, double* fib);
/* interpolation of a lattice vector field v (N*d) at markers, eq. Interpolation */
int orc_interp(const orc_sim* s, int n, const double* X, const double* v, double* U);

#ifdef __cplusplus
}
#endif
#endif
