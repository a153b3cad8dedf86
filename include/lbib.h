/*
 * lbib.h -- C ABI of the MI355X (gfx950) ternary free-energy lattice
 * Boltzmann + immersed-boundary library.
 *
 * Method: Pepona, Shek, Semprebon, Krueger, Kusumaatmaja, "Modelling ternary
 * fluids in contact with elastic membranes".  A simulation holds a lattice of
 * three population sets f, g, h (Sec. 3.1) and any number of closed elastic
 * membranes made of Lagrangian markers (Sec. 3.2), coupled by Peskin's
 * four-point kernel (Sec. 3.3).  One step advances both by one time unit.
 *
 * Conventions (all entry points)
 *   - Node (x, y, z) has linear index x + nx*(y + ny*z); x is periodic; y (and
 *     z in 3D) are periodic or bounded by half-way bounce-back walls at -1/2
 *     and n-1/2.  Marker coordinates are lattice units, node (x,y) at (x,y).
 *   - Memory.  The caller owns every buffer.  Device memory: one workspace of
 *     lbib_workspace_bytes() bytes, 256-byte aligned, kept alive and
 *     untouched until lbib_destroy.  The library never allocates device
 *     memory.  Host arrays passed in are copied before the call returns;
 *     host arrays passed out are filled by the callee.
 *   - Streams.  hip_stream is a hipStream_t (NULL = the default stream).
 *     lbib_step only enqueues work; the getters synchronise the stream.
 *     With lbib_set_overlap(s, 1) a D2Q9 step also uses a second stream
 *     that the handle creates on first use and releases in lbib_destroy;
 *     every step still ends ordered on hip_stream.
 *     One host thread per handle; calls on one handle must not overlap.
 *   - Errors.  Every call returns an lbib_status; no exception crosses the
 *     ABI.  A failed call leaves the handle as it was, except LBIB_EHIP,
 *     after which the handle should be destroyed.
 *   - Determinism.  For fixed inputs and build, results are bitwise
 *     reproducible on the same GPU: the only atomics are integer additions
 *     of fixed-point values.
 */
#ifndef LBIB_H
#define LBIB_H
#include <stddef.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbib_sim lbib_sim;

typedef enum {
  LBIB_OK = 0,
  LBIB_EINVAL = -1,      /* bad argument or parameter                          */
  LBIB_ENOMEM = -2,      /* workspace too small, or a capacity exceeded         */
  LBIB_EHIP = -3,        /* a HIP runtime call failed                           */
  LBIB_ENONFINITE = -4,  /* a non-finite value was found by lbib_check          */
  LBIB_EUNSTABLE = -5,   /* a force left the fixed-point range                  */
  LBIB_ESTATE = -6       /* call out of order (e.g. step before set_fields)     */
} lbib_status;

enum { LBIB_D2Q9 = 0, LBIB_D3Q19 = 1 };
/* population storage.  FP32/FP64 keep f_i - w_i, g_i and h_i (Sec. 3.1 EDF:
   f is near its weight, g and h moving populations near zero); FP32 keeps
   the rest populations g_0 and h_0 (which carry phi and psi) in FP64.  The
   16-bit forms keep the moving populations in half or bfloat16 (scaled by
   2^10), f_0 - w_0 in FP32 and g_0, h_0 in FP64; each moving population's
   rounding goes into its node's rest population, so every set's mass is
   conserved. */
enum { LBIB_FP32 = 0, LBIB_FP16 = 1, LBIB_BF16 = 2, LBIB_FP64 = 3 };

typedef struct {
  int lattice;              /* LBIB_D2Q9 (Sec. 3.1) or LBIB_D3Q19                     */
  int nx, ny, nz;           /* nz = 1 for D2Q9                                        */
  int wall_y, wall_z;       /* 0 periodic, 1 bounce-back walls                        */
  double tau, tau_phi, tau_psi;   /* relaxation times, eq. RelaxationTimes (> 1/2)    */
  double gamma_phi, gamma_psi;    /* Gamma of g^eq, h^eq, eq. EDF                     */
  double kappa[3];          /* kappa_1..3 of eq. LandauFE                             */
  double alpha;             /* interface width of eq. LandauFE                        */
  double kappa_c;           /* coupling strength of eq. CouplingE                     */
  double r_cut;             /* coupling band: beyond this distance from a membrane,
                               the profile I of eq. Iprofile is exactly 0 or 1 and the
                               node adds no coupling force; <= 0 selects 17 alpha     */
  int storage;              /* LBIB_FP32, LBIB_FP16, LBIB_BF16 or LBIB_FP64           */
  int max_markers;          /* capacity: markers over all membranes                   */
  int max_elems;            /* capacity: triangles over all 3D membranes              */
  int max_membranes;        /* capacity: membranes                                    */
} lbib_params;

typedef struct {
  double mass[3];           /* sum over nodes of C1, C2, C3 (conserved)                */
  double F_bulk;            /* sum kappa_m/2 C_m^2 (1 - C_m)^2, eq. LandauFE            */
  double F_grad;            /* sum alpha^2 kappa_m/2 |grad C_m|^2, eq. LandauFE         */
  double E_c;               /* kappa_c/2 sum (psi - I)^2, eq. DiscreteCE               */
  double E_s, E_b;          /* membrane strain and bending, eqs. DiscreteSE/BE         */
  double E_kin;             /* 1/2 sum rho |u|^2 with the bare velocity u               */
  double p_ideal;           /* sum c_s^2 rho ln rho, the ideal-gas term of LandauFE
                               (with component densities c_s^2 (M1+M2)/2 n ln n,
                               n = C1 + C2 + C3; lbib_set_densities)                  */
} lbib_energies;

/* Device bytes needed for a simulation with these parameters and capacities. */
int lbib_workspace_bytes(const lbib_params* p, size_t* bytes);

/* Create a simulation in the caller's workspace (see Conventions). */
int lbib_create(const lbib_params* p, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                lbib_sim** out);

/* Add a closed membrane (Sec. 3.2).  2D: a ring of n_nodes markers, segment l
   joining markers l and l+1 (n_elems = 0, conn = NULL), counter-clockwise or
   clockwise.  3D: a closed triangle mesh, conn = 3*n_elems vertex ids.
   X: host, n_nodes*d doubles.  Rest lengths are the initial edge lengths.
   kappa_s, kappa_b: the moduli of eqs. StretchingE, BendingE.
   Must precede lbib_set_fields.  *membrane_id receives 0, 1, 2, ... */
int lbib_add_membrane(lbib_sim* s, int n_nodes, const double* X, int n_elems, const int* conn,
                      double kappa_s, double kappa_b, int* membrane_id);

/* Replace the rest lengths of membrane id (host array): 2D, one per
   segment l -> l+1 in marker order; 3D, one per mesh edge, edges ordered by
   (smaller vertex index, larger vertex index).  By default the rest lengths
   are those of the configuration given to lbib_add_membrane (the reference
   state of the strain energy, eq. DiscreteSE).  LBIB_EINVAL for a length
   that is not positive and finite. */
int lbib_set_rest(lbib_sim* s, int id, const double* rest);

/* Strain law of membrane id (the paper's law and the two hyperelastic laws it
   names as alternatives).  Per segment the strain energy is W(lam) times the
   rest length, lam = length / rest length:
     0 (default)  ks/2 (lam - 1)^2, eq. DiscreteSE
     1            ks/8 (lam - 1/lam)^2, the neo-Hookean membrane law
                  G/2 (l1^2 + l2^2 + (l1 l2)^-2 - 3) at plane strain (l2 = 1)
                  with G = ks/4
     2            ks/8 (lam^2 - 1)^2, the Skalak law G/4 (I1^2 + 2 I1 - 2 I2
                  + C I2^2) at plane strain with G (1 + C) = ks/2
   All three have the same small-strain stiffness ks.  On a D3Q19 mesh, law 0
   is the edge-spring law and laws 1 and 2 replace the springs by the
   membrane laws per triangle: each flat triangle maps linearly from its rest
   shape (its three rest edge lengths, lbib_set_rest) to its current one, with
   I1 = l1^2 + l2^2 and J = l1 l2 = area / rest area, energy rest area x
   G/2 (I1 + J^-2 - 3) (neo-Hookean) or G/4 ((I1-2)^2 + 2 (I1-2) - 2 (J^2-1)
   + (J^2-1)^2) (Skalak, C = 1), shear modulus G = ks; bending is unchanged.
   The forces are minus the energy's gradient and the energies enter
   lbib_energy's E_s.  Takes effect at the next step.  Synchronises.
   LBIB_EINVAL for another law, an unknown id or a batch handle. */
int lbib_set_membrane_law(lbib_sim* s, int id, int law);

/* Initial macroscopic fields (host, N doubles each; uz may be NULL in 2D and
   ux, uy may be NULL for a fluid at rest).  Builds the equilibrium
   populations of eq. EDF, with the chemical potentials of Appendix A taken
   from these fields and the membranes added so far. */
int lbib_set_fields(lbib_sim* s, const double* rho, const double* phi, const double* psi,
                    const double* ux, const double* uy, const double* uz);

/* Enqueue n_steps time steps on the stream.  Each step: moments, coupling
   profile I(X(t)) and coupling forces, chemical potentials (Appendix A),
   membrane forces (eq. DiscreteTF), spreading (eq. Spreading), fused
   collide + stream of f, g, h (eq. LBE), interpolation of the velocity at
   t+1 (eq. Interpolation) and the Euler marker update (eq. UpdatedXl). */
int lbib_step(lbib_sim* s, int n_steps);

/* Fields at the current time (host, N doubles each, any may be NULL):
   rho, C1 = (rho+phi-psi)/2, C2 = (rho-phi-psi)/2, C3 = psi
   (eq. VariableTransform) and the bare velocity u = sum c_i f_i / rho
   (eq. MomentsDFs).  Synchronises. */
int lbib_get_fields(lbib_sim* s, double* rho, double* c1, double* c2, double* c3, double* ux,
                    double* uy, double* uz);

/* Markers of membrane id (host, n_nodes*d doubles each, any may be NULL):
   positions X, the velocity U of the last update and the total force F of
   the last step.  Synchronises. */
int lbib_get_membrane(lbib_sim* s, int id, double* X, double* U, double* F);

/* Energies and conserved sums at the current time, FP64.  Synchronises. */
int lbib_energy(lbib_sim* s, lbib_energies* out);

/* Finiteness check of the populations (FP64 sums): LBIB_ENONFINITE when a
   population is NaN or infinite; LBIB_EUNSTABLE when, during the last steps,
   a marker force left the fixed-point range, a membrane's grown box (box +
   max(r_cut + 1, 3) each side) was as wide as a period, or a tile of the
   coupling pass lay within reach (r_cut + 1) of more membranes than it keeps
   band data for (four in 2D, two in 3D; then the excess membranes' coupling
   forces on that tile are lost).  Synchronises. */
int lbib_check(lbib_sim* s);

/* Device view of an internal array for zero-copy inspection:
   field 0: population buffer holding the current state, 1: coupling profile
   I (valid on tiles near membranes), 2: marker positions (3 doubles per
   marker).  *elems receives the element count. */
int lbib_device_view(lbib_sim* s, int field, void** dev_ptr, size_t* elems);

/* Checkpoint: lbib_save(s, NULL, &bytes) reports the size; with a buffer of
   at least that size it writes a header (a tag, the step counter, the marker
   and membrane counts, nx, ny, nz, Q, the storage format, the force form and
   the population bytes), then the populations and the markers' X, U, F.
   lbib_load restores a checkpoint taken from a simulation created with the
   same parameters and membranes; LBIB_EINVAL (and the handle unchanged) when
   any header word but the step counter differs from the handle's, or the
   buffer is shorter than the checkpoint.  Both synchronise. */
int lbib_save(lbib_sim* s, void* host_buf, size_t* bytes);
int lbib_load(lbib_sim* s, const void* host_buf, size_t bytes);

/* Kernel timing.  lbib_timing_enable(s, mask) clears the counters and
   records HIP events on the stream around the phases of every following step
   whose bit is set in mask (bit k = phase k below; 0 turns timing off);
   lbib_timing_read synchronises and returns, for n <= 4 phases, the summed
   milliseconds of [0] the fused lattice kernel, [1] the coupling profile
   and tile map, [2] membrane forces and spreading, [3] interpolation and
   marker update, and in *steps the number of steps timed. */
int lbib_timing_enable(lbib_sim* s, int on);
int lbib_timing_read(lbib_sim* s, double* ms, int n, int* steps);

/* Launch shape of the fused lattice kernel (a tuning knob; results do not
   depend on it): D2Q9, block_x lanes per workgroup (64, 128, 192 or 256;
   block_x - 4 interior columns); D3Q19, block_x the x extent of a
   workgroup's tile of 256 nodes (16, 32 (the default) or 64; the y extent
   is 256 / block_x); seg rows (D3Q19: planes) per workgroup, nxcd the number of L2 domains
   workgroups are dealt to in turn, ring the rows held in registers (3, or 4
   to load the next row while the current ones are computed).  0 keeps the
   current value; seg = -1 returns to the automatic choice (as many
   workgroups as fit on the GPU at once, so none waits for a second round),
   nxcd = -1 to the automatic dealing (eight domains, the XCDs of the
   MI355X, so that workgroups sharing halo rows or lines meet in one L2).  A value
   reported as 0 means automatic.  Invalid values change nothing. */
int lbib_set_launch(lbib_sim* s, int block_x, int seg, int nxcd, int ring);
int lbib_get_launch(const lbib_sim* s, int* block_x, int* seg, int* nxcd, int* ring);

/* D2Q9 step order (a scheduling knob; results are bitwise the same either
   way): with on = 1 the lattice regions whose workgroups read no membrane
   field (no active tile within their rows and lanes) are updated on a
   second stream, created by the library on first use and owned by the
   handle, while the profile and force kernels of Sec. 3.3 run on the
   simulation's stream; the regions next to the membranes follow them, and
   the step ends with the simulation's stream waiting for the second one.
   on = 0 (the default) runs the whole step on the simulation's stream;
   on = -1 selects the library's choice, which is 0 (the passes share the
   memory bandwidth, so the gain is a few per cent).  No effect on D3Q19
   simulations.  Both force forms.  Batch handles and members return
   LBIB_EINVAL, as do other values of on. */
int lbib_set_overlap(lbib_sim* s, int on);

/* D2Q9 form of the thermodynamic force of eq. ForceFE (Sec. 3.1).  form = 1
   (the default): the divergence form, -div P' - psi grad kappa_c (psi - I),
   with P' the non-ideal part of the pressure tensor of Appendix A (the bulk
   pressure sum_m C_m f_m' - f_m of eq. LandauFE plus its gradient terms
   alpha^2 kappa_m (grad C_m grad C_m - (|grad C_m|^2/2 + C_m lap C_m) I)).
   form = 0: the potential form of eq. GradPT, -rho grad mu_rho - phi grad
   mu_phi - psi grad mu_psi, with the coupling term of eq. CouplingE inside
   mu_psi.  Both use the isotropic stencils of the fused step and agree to
   second order in the grid spacing; the divergence form conserves the
   lattice momentum of the thermodynamic force exactly, the potential form
   only to the discretisation error, and on long runs (a liquid lens beyond
   about 30 000 steps) the potential form grows a slow mirror-symmetric flow
   that the divergence form does not have.  Takes effect at the next
   lbib_step.  On a batch handle the form applies to every member (the next
   step captures the batch's graphs again).  LBIB_EINVAL for other values,
   D3Q19 simulations and batch members. */
int lbib_set_force_form(lbib_sim* s, int form);

/* Coupling-profile search (a scheduling knob; results are bitwise the same
   either way).  on = 1 (the default): every node keeps, for up to two
   membranes near it, the closest membrane element found by the last full
   search (D2Q9: a ring segment; D3Q19: a triangle) and a lower bound on the
   distance of the elements farther off (D2Q9: more than eight segments
   along the ring; D3Q19: sharing no vertex with it), or, beyond the band,
   its side and a lower bound on its distance.  While the markers have not
   moved enough to break that bound (the library tracks the largest marker
   step of each membrane), the next step re-evaluates only the nearby
   elements, exactly, instead of searching.  on = 0 searches every step.  On
   a batch handle it applies to every member.  LBIB_EINVAL for other
   values. */
int lbib_set_coupling_cache(lbib_sim* s, int on);

/* Uniform external force density f_ext of eq. ForcingTermLBE (Sec. 3.1),
   added to the force of every node in every following step (the paper's
   runs have f_ext = 0, the default).  It enters the exact-difference forcing
   and the velocities of eqs. VelCorrection and ActualFluidVel like the other
   forces, so a uniform fluid gains f_ext of momentum per step.  fz must be 0
   for D2Q9.  Works on a simulation or a batch member (the batch then
   rebuilds its tables at the next step).  LBIB_EINVAL for non-finite values,
   fz != 0 in 2D, or a batch handle. */
int lbib_set_external_force(lbib_sim* s, double fx, double fy, double fz);

/* Component densities M_1, M_2, M_3 (the weights of eq. MassDensity,
   Sec. 2.1; the paper's model takes all three equal to 1, the default, and
   names unequal densities as its extension in Sec. 5).  rho is then the mass
   density sum_m M_m C_m while phi = C1 - C2 and psi = C3 keep their meaning
   (eq. VariableTransform), so the concentrations are a linear map of
   (rho, phi, psi), the chemical potentials of Appendix A follow through the
   transpose of that map, and the pressure tensor's gradient part takes its
   congruent kappa matrix.  The lattice carries the ideal-gas pressure of the
   number density n = sum_m C_m, c_s^2 (M_1 + M_2)/2 n, through a shift of
   f_i^eq that leaves its zeroth and first moments unchanged.  The
   concentrations lbib_get_fields returns, the masses and energies of
   lbib_energy (p_ideal becomes c_s^2 (M_1 + M_2)/2 sum n ln n) and
   lbib_set_fields' rho all use the mass density.  D2Q9 and D3Q19; call it
   before lbib_set_fields.  Works on a simulation or a batch member.
   LBIB_EINVAL for a value that is not finite and positive, or a batch
   handle; LBIB_ESTATE once the fields are set.  The checkpoint header
   records the densities, and lbib_load refuses a state saved with others. */
int lbib_set_densities(lbib_sim* s, double m1, double m2, double m3);

/* Number of completed steps. */
long long lbib_steps_done(const lbib_sim* s);

/* Failure injection for tests: write value into population entry idx of
   the current buffer (field 0) or marker coordinate idx (field 2). */
int lbib_debug_poke(lbib_sim* s, int field, long long idx, double value);

const char* lbib_strerror(int status);
/* Frees the handle (not the workspace).  A batch member is freed with its
   batch; destroying the member alone does nothing. */
void lbib_destroy(lbib_sim* s);

/* ------------------------------------------------------------------------
   Batches: n independent D2Q9 simulations (FP32 storage, n <= 256) in one
   workspace, stepped together.  Each phase of a step is one launch over all
   members (the lattice update one launch per size class: lattice width
   <= 128, <= 256, larger), and the step is captured once per buffer parity
   in a hipGraph and replayed (on a stream that can be captured, i.e. not
   the legacy default stream; otherwise the launches are enqueued directly).
   Every member gives the same results, bit for bit, as the same
   simulation created alone.
   ------------------------------------------------------------------------ */

/* Device bytes for a batch of params[0..n-1] (each as for lbib_create). */
int lbib_batch_workspace_bytes(int n, const lbib_params* params, size_t* bytes);

/* Create the batch in the caller's workspace.  LBIB_EINVAL for n outside
   [1, 256], a D3Q19 or non-FP32 member, or invalid parameters. */
int lbib_batch_create(int n, const lbib_params* params, void* dev_workspace, size_t ws_bytes,
                      void* hip_stream, lbib_sim** out_batch);

/* Handle of member k (owned by the batch): lbib_add_membrane,
   lbib_set_fields, lbib_get_fields, lbib_get_membrane, lbib_energy,
   lbib_save/lbib_load and lbib_check work on it as on a simulation created
   alone; lbib_step on a member is LBIB_ESTATE.  lbib_step(batch, n)
   advances every member n steps (all members must have their fields set);
   lbib_check(batch) checks every member.  Per-simulation calls on the
   batch handle itself return LBIB_EINVAL. */
int lbib_batch_member(lbib_sim* batch, int k, lbib_sim** member);

/* Lattice-kernel shape of size class size_class (0: width <= 128, 1:
   <= 256, 2: wider; -1: all): lanes per workgroup (64, 128, 192, 256), rows per
   work item (-1: automatic, one resident round of the class's items) and
   register ring depth (3 or 4); 0 keeps a value.  get_launch also returns
   the number of members in the class, and the rows in use once the batch
   has stepped. */
int lbib_batch_set_launch(lbib_sim* batch, int size_class, int block_x, int seg, int ring);
int lbib_batch_get_launch(lbib_sim* batch, int size_class, int* block_x, int* seg, int* ring,
                          int* members);

/* Graph replay on (1, the default) or off (0: direct launches); on < 0
   leaves it.  *active (may be NULL) is 1 when the last step replayed a
   graph. */
int lbib_batch_graph(lbib_sim* batch, int on, int* active);

/* ------------------------------------------------------------------------
   Warm-start network (not part of the paper's method: a learned initial
   guess of a 2D capsule's equilibrium shape; the plain cold start stays the
   reference).  A fully connected FP32 map 6 -> 128 -> 128 -> 32 with GELU
   (z Phi(z), Phi by erff) after both hidden layers; parameters in one array
   of lbib_mlp_param_count() floats: W1 [128][6], b1 [128], W2 [128][128],
   b2 [128], W3 [32][128], b3 [32] (row-major, output index first).  Inputs
   x [B][6] and targets t [B][32] are device arrays; the loss is
   sum (y - t)^2 / (2 B).  Training is deterministic (fixed-order sums).
   ------------------------------------------------------------------------ */
typedef struct lbib_mlp lbib_mlp;

int lbib_mlp_param_count(void);
/* Device bytes for batches of up to batch_max rows. */
int lbib_mlp_workspace_bytes(int batch_max, size_t* bytes);
int lbib_mlp_create(int batch_max, void* dev_workspace, size_t ws_bytes, void* hip_stream, lbib_mlp** out);
/* Host parameter arrays; set_params also clears the Adam moments and step
   count.  LBIB_EINVAL for non-finite values. */
int lbib_mlp_set_params(lbib_mlp* h, const float* host_params);
int lbib_mlp_get_params(lbib_mlp* h, float* host_params);
/* y_dev [B][32] = network(x_dev [B][6]), 1 <= B <= batch_max; enqueued. */
int lbib_mlp_forward(lbib_mlp* h, const float* x_dev, int B, float* y_dev);
/* Loss (may be NULL) and its gradient with respect to the parameters
   (host array, may be NULL); synchronises when either is asked for. */
int lbib_mlp_gradient(lbib_mlp* h, const float* x_dev, const float* t_dev, int B, double* loss,
                      float* grad_host);
/* One Adam step (bias-corrected moments) on the batch; loss (may be NULL)
   is that of the parameters before the step. */
int lbib_mlp_adam_step(lbib_mlp* h, const float* x_dev, const float* t_dev, int B, float lr, float beta1,
                       float beta2, float eps, double* loss);
void lbib_mlp_destroy(lbib_mlp* h);

/* Forward pass of the network without a workspace, for callers that cannot
   allocate device memory (code under graph capture, serving loops, hosts
   that forbid allocation): the same kernels and results as
   lbib_mlp_forward.  params_dev holds the lbib_mlp_param_count() parameters
   (device, the layout above), x_dev [B][6] and y_dev [B][32] are device
   arrays owned by the caller.  The hidden activations go to a fixed device
   array of the library, 2 x 4096 x 128 floats (4 MiB), which each GPU the
   library runs on holds until the process ends; its address is looked up on
   the first call made with that device current.  1 <= B <= 4096: LBIB_ENOMEM
   for B > 4096, LBIB_EINVAL for B < 1 or a null pointer.  Enqueued on
   hip_stream (NULL = the default stream); allocates nothing and does not
   synchronise.  All calls on one GPU share the array (it keeps the last
   call's activations): calls that overlap in time on one GPU race, so keep
   them on one stream or otherwise ordered. */
int lbib_mlp_forward_noalloc(const float* params_dev, const float* x_dev, int B, float* y_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
