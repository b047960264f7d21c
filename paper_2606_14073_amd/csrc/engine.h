// engine.h -- device data of one batch of replicas and the kernel launchers.
#pragma once

#include "common.h"

namespace nep {

constexpr int MAXFE = 64;     // listed spin-carrying neighbours kept for the spin couplings
constexpr int RCOEF = 4 * NB; // per-atom contracted radial-set coefficients
constexpr int MCOEF = 3 * NB; // per-spin-carrier contracted magnetic pair coefficients

// flags[] words
enum { F_REBUILD = 0, F_OVERFLOW = 1, F_COLOUR = 2, F_NONFINITE = 3, NFLAGS = 8 };

// Atoms of all resident replicas, concatenated: [0, N_fe) are spin-carrying
// (species 0) atoms of every replica in replica order, [N_fe, N) the others.
// Slot-major neighbour arrays are indexed [slot * N + atom].
struct Sys {
    int N, N_fe, n_rep, n_cells;
    int mag;               // 1: spin-aware model; 0: structural-only (no spin work, N_fe = species-0 count)
    const int *rid;        // [N]
    const int *orig;       // [N] index in the replica's caller order
    RepDev *rep;           // [n_rep]
    d4 *pos, *vel, *spin, *force, *field, *pos_ref, *spin_n, *spin_hat, *eta;
    // self-consistent midpoint: iterate x, previous residual and sweep result,
    // difference ring [depth][N_fe] (mixing only), Gram partials, decisions
    d4 *sc_x, *sc_f, *sc_g, *sc_dF, *sc_dG;
    double *sc_part, *sc_out;
    const int *colour;     // [N] colour on spin carriers, -1 elsewhere
    const int *col_idx;    // [N_fe] spin carriers grouped by colour
    const int *colpos;     // [N_fe] position of each spin carrier in col_idx
    const int *col_rid;    // [N_fe] replica of each entry of col_idx
    int *nbrR, *cntR, *cntFeR, *revR;
    int *nbrA, *cntA, *cntFeA, *revA, *a2r;
    int *cell_of, *cell_cnt, *cell_start, *cell_fill, *cell_atoms;
    int *flags;
};

// Device copy of a model, one array per arithmetic type: c^R, c^A, c^ex,
// c^dm, c^an, c^si, c^sa, W0 [2][DP][NH] (transposed, zero padded), b0, w1,
// b1, then the optional short-range term at M_ZBL: K Z_i Z_j and the inverse
// screening length 1/a for each pair type tau = 2 t_i + t_j, r_inner,
// r_outer, pi / (r_outer - r_inner), and 1 when the term is on (else 0).
constexpr int M_ZBL = 324 + 252 + 4 * 324 + 252 + 2 * DP * NH + 2 * NH + 2 * NH + 2;
constexpr int MODEL_DEV = M_ZBL + 12;

template <typename real>
struct ModelDev {
    const real *cR, *cA, *cEX, *cDM, *cAN, *cSI, *cSA;   // [4][n][9]
    const real *W0;        // [2][64][DP], zero padded
    const real *b0, *w1, *b1;
};

template <typename real>
struct Work {
    real *q, *Fp, *Ei, *AB;     // [N][DP], [N][DP], [N], [N][NA][NAB]
    real *rcoef;                // [4][N][NB]: radial (blocks 0, 1) and single-ion (2, 3) coefficients contracted with the atom's Fp, per neighbour species
    real *mcoef;                // [N_fe][3 NB]: exchange, DMI, anisotropic-exchange coefficients contracted with the atom's Fp
    real *ownM;                 // [N_fe][6]: magnetic-pair sum_j dE_i/dd_ij, dE_i/ds_i
    real *pbA;                  // angular pair records [MAXA][N][4]: dE_i/dd_ij, h_ij, stored likewise
    real *ownR;                 // [N][6]: radial and single-ion sum_j dE_i/dd_ij, dE_i/ds_i
    real *ownA;                 // [N][6]: angular-set sum_j dE_i/dd_ij, sum_j h_ij s_j
    real *csa;                  // [MAXFE][N_fe]: spin-angular part of a_ij at j's slot in i's rc_R row (atom order)
    real *cpl;                  // [MAXFE][N_fe][6]: J, D, K, rhat (colour-list order)
    real *selfc;                // [N_fe][8]: A_i (xx yy zz xy xz yz), o_i (colour-list order)
    int *cpl_j;                 // [MAXFE][N_fe]: neighbour of each coupling (colour-list order)
    int *cpl_n;                 // [N_fe]: couplings inside rc_R per spin (colour-list order)
};

// ---- launchers (kernels_*.hip) ----
void launch_skin_check(const Sys &S, hipStream_t st);
void launch_rebuild(const Sys &S, double r_listR, double r_listA, hipStream_t st);

// forward-pass modes: the full evaluation, the spin step's first pass at the
// mid positions, and its later passes at the same positions
enum { PASS_FULL = 0, PASS_SPIN = 1, PASS_SPIN_REUSE = 2 };

template <typename real>
void launch_desc_radial(const Sys &S, const ModelDev<real> &M, const Work<real> &W, const d4 *spin, int mode,
                        hipStream_t st);
template <typename real>
void launch_desc_angular(const Sys &S, const ModelDev<real> &M, const Work<real> &W, const d4 *spin, int mode,
                         hipStream_t st);
template <typename real>
void launch_mlp(const Sys &S, const ModelDev<real> &M, const Work<real> &W, int mode, hipStream_t st);
template <typename real>
void launch_bwd_radial(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st);
template <typename real>
void launch_bwd_angular(const Sys &S, const ModelDev<real> &M, const Work<real> &W, int species,
                        hipStream_t st);   // one launch: species 0 (spin carriers) or 1
template <typename real>
void launch_gather(const Sys &S, const Work<real> &W, hipStream_t st);
template <typename real>
void launch_assemble_coef(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st);
template <typename real>
void launch_assemble_pairs(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st);
template <typename real>
void launch_sweep(const Sys &S, const Work<real> &W, const int *col_ptr_host, int n_colours, hipStream_t st);

void launch_kick(const Sys &S, hipStream_t st);
void launch_drift(const Sys &S, hipStream_t st);
void launch_langevin(const Sys &S, hipStream_t st);
void launch_spin_prep(const Sys &S, hipStream_t st);
void launch_spin_restore(const Sys &S, hipStream_t st);
void launch_spin_mid(const Sys &S, hipStream_t st);
void launch_step_end(const Sys &S, hipStream_t st);
// rep[r].active = act[r] for every r < n with act[r] >= 0
void launch_set_active(RepDev *rep, const int *act, int n, hipStream_t st);
// re-layout: row k of the five state arrays takes row src[k] of the staged old
// arrays (array a at stage + a n_old); src[k] < 0 leaves row k alone
void launch_gather_state(const d4 *stage, size_t n_old, const int *src, int n, d4 *pos, d4 *vel, d4 *spin, d4 *force,
                         d4 *field, hipStream_t st);
// self-consistent midpoint: residual of the pass, per replica converged or
// not, and with depth > 0 the mixing coefficients; sc_out[0] = replicas still
// iterating, sc_out[1] = largest change, sc_out[2] = columns used, then gam
constexpr int SC_OUT = 12;
constexpr int SC_MAXD = 8;                                     // deepest mixing history
constexpr int SC_NK = SC_MAXD * (SC_MAXD + 1) / 2 + SC_MAXD;   // Gram entries + right-hand side
int sc_part_blocks(int n_fe);
void launch_sc_check(const Sys &S, int pass, int depth, double reg, int k_corr, hipStream_t st);
void launch_sc_mix(const Sys &S, int pass, int depth, hipStream_t st);

// per-replica fixed-order reductions: out[r][NOBS]: E_nep, E_kin, E_z,
// Ts_num, Ts_den, Mx, My, Mz, sum |s|, rotations stopped at the cap, and
// last the count of non-finite atoms
constexpr int NOBS = 11;
struct Chunk {
    int rid, begin, end;
};
template <typename real>
void launch_observe(const Sys &S, const Work<real> &W, const Chunk *chunks, int n_chunks,
                    const int *chunk_ptr, double *partial, double *out, hipStream_t st);

}  // namespace nep
