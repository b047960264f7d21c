/*
 * nepspin.h -- C ABI of the MI355X spin-lattice NEP library.
 *
 * The library evaluates a spin-aware neuro-evolution potential E(R,S) and
 * advances coupled lattice/spin dynamics with it on one AMD Instinct MI355X
 * (gfx950). Method: "Extreme-Scale Atomistic Simulation of Real-Temperature
 * Magnetic Skyrmion Dynamics by Coupled Spin-Lattice Modeling":
 *   - unified energy surface E(R,S) with lattice and spin driving terms,
 *     Sec. 5.2 "Unified spin-lattice execution";
 *   - spin-aware local descriptor (structural radial/angular channels plus
 *     onsite, pairwise exchange/DMI/anisotropic/single-ion, and spin-weighted
 *     angular channels), Sec. 5.1 "A spin-aware local descriptor pipeline" and
 *     "Implementation-oriented descriptor organization";
 *   - Chebyshev radial basis of size 8, Sec. 5.2 "SVE2 predicated
 *     vectorization" and "SME three-stage pipeline";
 *   - symplectic spin-lattice integrator with a predictor-corrector spin
 *     update scheduled last, Sec. 3 and Sec. 5.1 "Self-consistent midpoint
 *     spin update"; finite-temperature baths on both lattice and spins, Sec. 8.
 *
 * Units: Angstrom, eV, fs, atomic mass units, K, Tesla. Spins are
 * dimensionless vectors (|s| = 1 on magnetic atoms); the effective field
 * H = -dE/ds is in eV. Species 0 (Fe) carries a spin, species 1 (Ge) does not:
 * spin rows of species-1 atoms are ignored (treated as zero) and their field
 * rows are returned as zero.
 *
 * Conventions for every call:
 *   - Return value: 0 (SL_OK) on success, a negative sl_status otherwise; the
 *     library never aborts or exits. sl_last_error() gives a message for the
 *     calling thread's last failure.
 *   - Ownership: the caller owns every array it passes. Inputs are copied
 *     before the call returns; outputs are written into caller buffers. Opaque
 *     handles are owned by the library and released only by the matching
 *     *_destroy call.
 *   - Atom order is the caller's order; any internal reordering is invisible.
 *   - Arrays are C-contiguous; "[n][3]" means 3 doubles per atom, atom-major.
 *   - Threading: an nep_model may be shared by several threads once created;
 *     an sl_sim must be used by one thread at a time; server calls are
 *     thread-safe.
 */
#ifndef NEPSPIN_H
#define NEPSPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SL_OK = 0,
    SL_E_INVALID = -1,    /* bad argument, size or hyper-parameter          */
    SL_E_OOM = -2,        /* device memory or HBM budget exceeded           */
    SL_E_BOX = -3,        /* periodic box edge < 2 (r_c^R + skin)           */
    SL_E_DEVICE = -4,     /* HIP runtime error                              */
    SL_E_NONFINITE = -5,  /* NaN/Inf in the state of a replica              */
    SL_E_NOTFOUND = -6,   /* unknown replica id                             */
    SL_E_BUSY = -7,       /* replica not finished yet                       */
    SL_E_OVERFLOW = -8,   /* neighbour list capacity exceeded               */
    SL_E_NOLIB = -9       /* no usable GPU / device code                    */
} sl_status;

/* Arithmetic of the potential (descriptor, read-out, backward, couplings).
 * Positions, velocities, spins, minimum-image displacements, spin rotations
 * and energy sums are FP64 in every mode. */
typedef enum {
    SL_FP64 = 0,          /* everything FP64                                */
    SL_FP32_MIXED = 1     /* potential in FP32, accumulated in FP32          */
} sl_precision;
/* Any other value is SL_E_INVALID. (A BF16 input->hidden contraction of the
 * read-out was measured at 3.7e-4 eV/atom and 1e-3 relative force error,
 * outside the FP32 bounds, and is not offered.) */

const char *sl_last_error(void);

typedef struct nep_model nep_model;
typedef struct sl_sim sl_sim;
typedef struct sl_server sl_server;

/* ---------------------------------------------------------------------- */
/* Model                                                                  */
/* ---------------------------------------------------------------------- */

/* Hyper-parameters of the spin-aware NEP. The library supports exactly:
 * n_max_R = 8 (9 radial-set functions), n_max_A = 6 (7 angular-set
 * functions), l_max = 4, basis_K = 8 (Chebyshev T_0..T_8), n_hidden = 64,
 * n_species = 2, rc_R = 6.0, rc_A = 4.5 (Angstrom); anything else is
 * SL_E_INVALID. */
typedef struct {
    int n_max_R, n_max_A, l_max, basis_K, n_hidden, n_species;
    double rc_R, rc_A;
    int structural;      /* 0: the spin-aware NEP below. 1: the structural-only
                            NEP it extends (Sec. 5.1: the magnetic groups augment
                            the structural channels): descriptor q^R (9) and
                            q^A (28), 5,570 parameters c^R[4][9][9],
                            c^A[4][7][9], then per species W0[64][37], b0[64],
                            w1[64], b1[1]. No spins: spin inputs are ignored,
                            fields are zero, a step is B A O A B, and
                            nep_spin_descriptors returns [n][37] arrays.       */
    /* Optional short-range repulsion (Sec. 6 includes an optional short-range
     * pair term in the modeled work of a step without giving its form; the
     * form here is the universal screened-Coulomb potential of Ziegler,
     * Biersack and Littmark):
     *   E_i += 1/2 sum_j V(r_ij),  V(r) = K Z_i Z_j / r * phi(r/a) * S(r),
     *   K = 14.399645 eV A, a = 0.8854 * 0.529177210903 A / (Z_i^0.23 + Z_j^0.23),
     *   phi(x) = 0.18175 e^{-3.19980x} + 0.50986 e^{-0.94229x}
     *          + 0.28022 e^{-0.40290x} + 0.02817 e^{-0.20162x},
     *   S(r) = 1 below sr_r_inner, (1 + cos(pi (r - sr_r_inner)/(sr_r_outer - sr_r_inner)))/2
     *          between, 0 from sr_r_outer on.
     * sr_Z[t] is the nuclear charge of species t. sr_r_outer = 0 turns the
     * term off; otherwise 0 < sr_r_inner < sr_r_outer <= rc_R and Z > 0 are
     * required (SL_E_INVALID). It adds to E, E_i and F only.              */
    double sr_Z[2];
    double sr_r_inner, sr_r_outer;
    /* Optional onsite moment-length term of the spin carriers, for spins of
     * variable length (Sec. 3: the integrator carries the longitudinal
     * fluctuation of the magnetic moment):
     *   E_i += moment_a |s_i|^2 + moment_b |s_i|^4   (species 0),
     * a Landau expansion whose minimum sits at |s|^2 = -moment_a/(2 moment_b);
     * it adds to E, E_i and H (H_i -= (2 moment_a + 4 moment_b |s_i|^2) s_i).
     * Both 0: off. moment_b < 0 (unbounded below) is SL_E_INVALID.         */
    double moment_a, moment_b;
} nep_spin_hparams;

/* params: 15,438 doubles in this order (tau = 2 t_i + t_j is the ordered
 * species pair of centre i and neighbour j):
 *   c^R[4][9][9], c^A[4][7][9], c^ex[4][9][9], c^dm[4][9][9], c^an[4][9][9],
 *   c^si[4][9][9], c^sa[4][7][9], then for species t = 0, 1:
 *   W0[64][102], b0[64], w1[64], b1[1].
 * Radial functions: f_k(r) = (T_k(x)+1)/2 * (1+cos(pi r/rc))/2 with
 * x = 2(r/rc-1)^2-1 for r < rc (zero beyond); g^X_n(r) = sum_k c^X[tau][n][k] f_k(r).
 * Descriptor q[102] of atom i (sums over neighbours within the channel's
 * cutoff, rc_R for R/ex/dm/an/si and rc_A for A/sa; j,k independent):
 *   0..8    q^R_n     = sum_j g^R_n(r_ij)
 *   9..36   q^A_{nl}  = sum_j sum_k g^A_n(r_ij) g^A_n(r_ik) P_l(rhat_ij.rhat_ik), at 9+4n+l-1
 *   37      q^os      = s_i.s_i
 *   38..46  q^ex_n    = sum_j g^ex_n (s_i.s_j)
 *   47..55  q^dm_n    = sum_j g^dm_n rhat_ij.(s_i x s_j)
 *   56..64  q^an_n    = sum_j g^an_n (s_i.rhat_ij)(s_j.rhat_ij)
 *   65..73  q^si_n    = sum_j g^si_n (s_i.rhat_ij)^2
 *   74..101 q^sa_{nl} = sum_j sum_k g^A_n(r_ij) g^sa_n(r_ik) (s_i.s_k) P_l(rhat_ij.rhat_ik)
 * Energy: E_i = b1 + sum_h w1_h tanh(b0_h + sum_d W0_hd q_d), E_NEP = sum_i E_i.
 * The model keeps a device copy of the parameters. */
int nep_model_create(const nep_spin_hparams *hp, const double *params, size_t n_params,
                     nep_model **out);
int nep_model_destroy(nep_model *m);

/* One system, caller-owned and read-only. types[n] in {0,1}; pos[n][3];
 * spin[n][3] (rows of species 1 ignored); box edges; pbc[a] = 1 for a
 * periodic axis (minimum image), 0 for a free axis. mu_s is the moment of a
 * species-0 atom in Bohr magnetons; B the applied field in Tesla (Zeeman
 * energy -mu_s mu_B B.s_i on species-0 atoms). */
typedef struct {
    int64_t n_atoms;
    const int32_t *types;
    const double *pos;
    const double *spin;
    double box[3];
    int32_t pbc[3];
    double mu_s;
    double B[3];
} sl_system_view;

/* Execution options. device_ptrs = 0: the output pointers of nep_spin_eval
 * are host memory. device_ptrs = 1: they are device memory of the current
 * HIP device. hip_stream: a hipStream_t, or NULL for the library's stream.
 * A NULL sl_exec means host pointers and the library's stream; calls return
 * after the results are in place. */
typedef struct {
    int device_ptrs;
    void *hip_stream;
} sl_exec;

/* Energy, forces and fields of one system (Sec. 5.2: one pass producing both
 * lattice and spin driving terms).
 *   energy[1]      : E_NEP + E_Zeeman (FP64 sum)
 *   energy_atom[n] : E_i (NEP part), or NULL
 *   force[n][3]    : F_i = -dE/dr_i, or NULL
 *   field[n][3]    : H_i = -dE/ds_i (+ mu_s mu_B B), species-0 rows; or NULL
 * The model keeps the device work arrays of its last evaluation (about
 * 13 KB per atom in FP64, 8 KB in FP32) for the next call of the same
 * precision; another precision, a system more than eight times smaller or
 * nep_model_destroy releases them. Calls on one model are serialised.
 * Errors: SL_E_INVALID (bad sizes/types), SL_E_BOX, SL_E_OVERFLOW (more than
 * 160 neighbours inside 6.5 A, 96 inside 5 A, or 64 species-0 neighbours of a
 * spin carrier inside 6.5 A), SL_E_OOM, SL_E_DEVICE. */
int nep_spin_eval(const nep_model *m, const sl_system_view *sys, sl_precision prec,
                  double *energy, double *energy_atom, double *force, double *field,
                  const sl_exec *ex);

/* Intermediate arrays of the same evaluation, for inspection: q[n][102]
 * (descriptor, caller order) and Fp[n][102] = dE_i/dq_i. Either may be NULL.
 * Same pointer rules and errors as nep_spin_eval. */
int nep_spin_descriptors(const nep_model *m, const sl_system_view *sys, sl_precision prec,
                         double *q, double *Fp, const sl_exec *ex);

/* nep_spin_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with every device buffer the evaluation needs
 * (state, neighbour lists, cells, descriptor/gradient work arrays,
 * reductions) carved from one static scratch array of 64 MiB that each GPU
 * the library runs on holds until the process ends. No hipMalloc, hipFree,
 * stream or event is created; work runs on ex->hip_stream (NULL: the null
 * stream) and the call returns after the results are in place.
 * Limit: the system must fit the 64 MiB, about 5,000 atoms in FP64 and 8,000
 * in FP32-mixed (dense crystal, about 13 and 8 KB per atom); a larger one
 * returns SL_E_OOM before any device work. Every call on one GPU shares its
 * array, which keeps the last call's contents (what must start at zero is
 * cleared on each call), so two calls that overlapped on one GPU would race:
 * the library serialises them within a process (each process has its own
 * array). Same arguments, outputs and other errors as nep_spin_eval. */
int nep_spin_eval_noalloc(const nep_model *m, const sl_system_view *sys, sl_precision prec,
                          double *energy, double *energy_atom, double *force, double *field,
                          const sl_exec *ex);

/* ---------------------------------------------------------------------- */
/* Spin-lattice integration                                               */
/* ---------------------------------------------------------------------- */

/* One step n -> n+1 is the symmetric splitting B A O S A B:
 *   B: v += (dt/2) kappa F/m;  A: r += (dt/2) v, wrapped into the box;
 *   O (ensemble = 1): v = c1 v + sqrt((1-c1^2) kappa kB T_n/m) xi, c1 = exp(-gamma_L dt);
 *   S: spin step at the mid positions: for p = 0..K_corr, the magnetic part of
 *      E is linearised with Fp taken at reference spins S_hat (S_hat = S^n for
 *      p = 0, then normalise((S^n + S^(p-1))/2)); from S^n, every spin of
 *      colour 0,1,..,C-1 and then C-1,..,0 takes an implicit-midpoint
 *      Rodrigues rotation over dt/2 with
 *        omega = (h + alpha_s xbar x h)/(1+alpha_s^2),
 *        h = H_lin(xbar) + mu_s mu_B B_n + eta_i,
 *        eta_i = sqrt(2 alpha_s kB T_n hbar/dt) xi_i (fixed for the step),
 *      the midpoint equation y = G(y) solved until max|G(y)-y| <= mid_tol
 *      or mid_cap iterations, the result being G(y) (Newton steps with a
 *      finite-difference Jacobian; mid_cap = 1 is the explicit rotation);
 *   A; then E, F, H at (R^{n+1}, S^{n+1}); B.
 * T_n = T0 + (T1-T0) min(n, n_ramp)/n_ramp and B_n likewise (constant T0, B0
 * when n_ramp = 0). xi are Philox4x32-10 normals keyed by seed, counted by
 * (atom index in the caller's order, step, stream 0 lattice / 1 spin).
 * kappa = 9.648533212e-3, kB = 8.617333262e-5 eV/K, hbar = 0.6582119569 eV fs,
 * mu_B = 5.7883818060e-5 eV/T, masses 55.845 (Fe) and 72.630 (Ge) u. */
typedef struct {
    double dt, T0, T1, B0[3], B1[3], alpha_s, gamma_L;
    int64_t n_ramp;
    int ensemble;        /* 0 NVE (no O step, alpha_s must be 0 for NVE spins), 1 Langevin */
    int K_corr;          /* number of corrector passes (0 = predictor only)  */
    double mid_tol;      /* per-spin midpoint tolerance, e.g. 1e-15           */
    int mid_cap;         /* per-spin cap on the iterations of the midpoint
                            equation, 1..1000 (1: the explicit rotation G(s)).
                            The solve is Newton's method, so it needs fewer
                            iterations than plain fixed-point iteration; the
                            result is defined up to mid_tol only when the
                            equation converged, which sl_observables.mid_capped
                            reports for every step                           */
    uint64_t seed;       /* Philox key                                        */
    double skin;         /* Verlet skin (A); lists rebuilt when an atom moved
                            more than skin/2 since the last build             */
    double sc_tol;       /* > 0: self-consistent midpoint (Sec. 5.1): pass p
                            sweeps from S^n at the midpoint of S^n and x^(p)
                            (x^(0) = S^n; plain iteration: x^(p) = S^(p-1));
                            passes repeat until max over spins of
                            |S^(p) - x^(p)| <= sc_tol (p >= 1) or p = sc_max.
                            K_corr is then not used. 0: off. Single-system
                            simulations only (sl_create); the host reads one
                            small decision per pass.                         */
    int sc_max;          /* cap on corrector passes when sc_tol > 0          */
    double mass[2];      /* per species (u); 0 = 55.845 (species 0), 72.630   */
    int sc_depth;        /* accelerated variant (Sec. 5.1), 0..8: the next
                            iterate mixes the last sc_depth residual
                            differences (Anderson); 0: plain iteration       */
    double sc_reg;       /* Tikhonov regularisation of the mixing, relative
                            to the mean diagonal of the residual Gram matrix */
    int longitudinal;    /* 1: spins of variable length (Sec. 3, longitudinal
                            fluctuation of the moment), Langevin dynamics
                              ds/dt = (h x s)/hbar + (gamma_lsf/hbar) h + xi,
                              <xi xi> = 2 gamma_lsf kB T_n/hbar (isotropic),
                            whose equilibrium density over vectors s is
                            exp(-E/kB T). Each colour visit of the sweep is
                            then L(dt/4) R(dt/2) L(dt/4): R the rotation
                            above with alpha_s = 0 and the midpoint taken at
                            length |s|, L the Euler-Maruyama step
                            s += (gamma_lsf t/hbar) h(s) + sqrt(2 gamma_lsf kB T_n t/hbar) xi
                            with h the frozen-Fp field at s (Philox streams
                            2 + 2v and 3 + 2v, v = 0 ascending, 1 descending
                            pass); reference spins are the plain average
                            (S^n + S^(p))/2. alpha_s must be 0 (the damping
                            is gamma_lsf). 0: unit spins as above.           */
    double gamma_lsf;    /* damping of the longitudinal dynamics (>= 0)      */
} sl_integrator_params;

typedef struct {
    int64_t step;
    double E_pot;        /* E_NEP (+ short-range and moment-length terms) at
                            the end of the step                              */
    double E_kin;
    double E_zeeman;
    double T_lattice;    /* 2 E_kin / (3 N kB)                               */
    double T_spin;       /* sum|s x H|^2 / (2 kB sum s.H) over spins          */
    double M[3];         /* mean spin                                         */
    int32_t spin_passes; /* sweeps of the spin step: K_corr + 1, or the number
                            the self-consistent iteration took               */
    int32_t mid_capped;  /* spin rotations of the step (all passes) whose
                            midpoint equation still missed mid_tol after
                            mid_cap iterations (0 when every one converged)  */
    double spin_change;  /* self-consistent: max |S^(p) - x^(p)| of the last
                            pass (x^(p): the spins whose midpoint it used);
                            0 otherwise                                      */
    double spin_length;  /* mean |s| over the spins                          */
} sl_observables;

/* Create a simulation of one system: copies the state to the device and
 * evaluates F^0. vel[n][3] may be NULL (zero). colour[n]: colour class
 * (0..C-1) of each species-0 atom and -1 elsewhere; NULL lets the library
 * colour greedily (graph r < r_c^R + skin + 0.5 A, atoms in caller order).
 * Two spins of one colour within r_c^R of each other would be updated at once
 * although coupled: SL_E_INVALID. The colouring is kept like a neighbour list:
 * whenever a list rebuild finds two same-colour spins within r_c^R + skin
 * (not yet coupled, and unable to come within r_c^R before the next rebuild),
 * the system stops after that step, its colouring is repaired at the current
 * positions (in caller order, a spin that shares its colour with a spin
 * within r_c^R + skin + 0.5 A takes the smallest colour none of those has;
 * the others keep theirs), and it goes on; the steps stay exact, only the
 * sweep order changes.
 * Errors: SL_E_INVALID, SL_E_BOX, SL_E_OOM, SL_E_OVERFLOW, SL_E_DEVICE. */
int sl_create(const nep_model *m, const sl_system_view *sys, const double *vel,
              const int32_t *colour, const sl_integrator_params *ip, sl_precision prec,
              sl_sim **out);

/* Advance n_steps steps. per_step_out[n_steps] receives the observables of
 * every step, or NULL. Errors: SL_E_NONFINITE (state not finite),
 * SL_E_OVERFLOW, SL_E_INVALID (colouring), SL_E_DEVICE. */
int sl_integrate_steps(sl_sim *s, int64_t n_steps, sl_observables *per_step_out);

/* Current colouring in caller order (colour[n], -1 on species 1; may be NULL)
 * and the number of colour repairs since creation (may be NULL). */
int sl_get_colour(const sl_sim *s, int32_t *colour, int64_t *n_recolour);

/* State in caller order: pos, vel, spin [n][3] (any may be NULL), step. */
int sl_get_state(const sl_sim *s, double *pos, double *vel, double *spin, int64_t *step);

/* Replace the state (checkpoint resume); F is re-evaluated. */
int sl_set_state(sl_sim *s, const double *pos, const double *vel, const double *spin, int64_t step);

int sl_destroy(sl_sim *s);

/* Kernel timing for measurement. When enabled for a kernel group, every
 * launch of that group inside sl_integrate_steps is bracketed by HIP events
 * on the simulation's stream; totals accumulate until read. Groups:
 *   0 descriptor (radial set)   1 descriptor (angular set)   2 read-out
 *   3 backward (radial set)     4 backward (angular set), species 0
 *   5 gather                    6 spin-coupling coefficients and spin-angular parts
 *   7 colour sweep              8 neighbour lists
 *   9 lattice half-steps, baths and reductions
 *  10 spin-pair coupling assembly
 *  11 backward (angular set), species 1
 * mask: bit g enables group g (0 disables timing). */
#define SL_NPROF 12
int sl_profile_enable(sl_sim *s, unsigned mask);

/* ms_total[SL_NPROF]: summed event time per group (ms); launches[SL_NPROF]:
 * number of timed launch groups. Either may be NULL. Resets the totals. */
int sl_profile_read(sl_sim *s, double *ms_total, int64_t *launches);

/* ---------------------------------------------------------------------- */
/* Replica serving                                                        */
/* ---------------------------------------------------------------------- */

typedef struct {
    size_t hbm_budget_bytes;   /* 0: free device memory minus 4 GiB            */
    int max_slots;             /* most replicas resident at once               */
    sl_precision precision;
    int steps_per_batch;       /* steps per batched launch sequence             */
    int K_corr;                /* corrector passes, common to all replicas     */
} sl_server_config;

typedef enum { SL_QUEUED = 0, SL_RUNNING = 1, SL_DONE = 2, SL_FAILED = 3 } sl_replica_state;

typedef struct {
    int state;                 /* sl_replica_state                              */
    int error;                 /* sl_status of a failed replica                 */
    int64_t steps_done, n_steps;
    double t_submit, t_admit, t_done;     /* seconds since server start        */
    double step_latency_p50, step_latency_p99;   /* seconds, over its steps     */
    int64_t n_latency_samples;
} sl_replica_status;

/* A server owns a worker thread that admits queued replicas while slots and
 * the HBM budget allow, keeps their state on the device, and advances all
 * resident replicas together in batched launches. Results of a replica do
 * not depend on which other replicas share the device. */
int sl_server_create(const nep_model *m, const sl_server_config *cfg, sl_server **out);

/* Device memory a replica of n_atoms is charged against the server's HBM
 * budget in the given precision (work arrays, lists, state; the same figure
 * sizes a single-system simulation). */
size_t sl_replica_bytes(int64_t n_atoms, sl_precision prec);

/* Queue a replica (inputs copied; colour may be NULL). ip->K_corr must equal
 * the server's. A replica may iterate the midpoint to a tolerance
 * (ip->sc_tol > 0) with plain iteration only (ip->sc_depth 0): each replica
 * stops on its own criterion, those with fixed corrector passes after their
 * K_corr, so the result is the same as alone or as a single-system
 * simulation; its observables report its own pass count and last change.
 * Errors: SL_E_INVALID, SL_E_BOX, SL_E_OOM (larger than the whole budget). */
int sl_replica_submit(sl_server *sv, const sl_system_view *sys, const double *vel,
                      const int32_t *colour, const sl_integrator_params *ip, int64_t n_steps,
                      uint64_t *id_out);

int sl_replica_poll(sl_server *sv, uint64_t id, sl_replica_status *out);

/* Final state of a finished replica (any pointer may be NULL); SL_E_BUSY
 * while it runs. obs receives its last step's observables. */
int sl_replica_fetch(sl_server *sv, uint64_t id, double *pos, double *vel, double *spin,
                     sl_observables *obs);

/* Block until every submitted replica is done or failed. */
int sl_server_drain(sl_server *sv);

/* Aggregate counters since creation: steps (batched launches), atom-steps,
 * busy seconds. Any pointer may be NULL. */
int sl_server_stats(sl_server *sv, int64_t *batched_steps, double *atom_steps, double *busy_s);

/* Host time between batches since creation: the number of re-layouts (an
 * admission, a retirement or a recolouring changed the resident set), the
 * seconds they took (state staging, list rebuild, evaluation of the new
 * replicas, checks), and the seconds of all gaps between the end of one
 * batch and the start of the next (re-layouts, retirement downloads, host
 * bookkeeping). Each gap is also counted in the latency of the first step of
 * the batch that follows it. Any pointer may be NULL. */
int sl_server_host_stats(sl_server *sv, int64_t *relayouts, double *relayout_s, double *gap_s);

int sl_server_destroy(sl_server *sv);

#ifdef __cplusplus
}
#endif

#endif
