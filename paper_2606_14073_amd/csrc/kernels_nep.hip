// kernels_nep.hip -- the spin-aware NEP on the device: descriptor, per-species
// read-out, backward pass (forces and effective fields) and the bilinear spin
// couplings of the frozen-Fp magnetic energy.
//
// Mapping. Radial-set work (radial, exchange, DMI, anisotropic, single-ion
// channels over the 6 A list) runs one lane per atom. Angular-set work
// (angular and spin-angular channels over the 4.5 A list) runs eight lanes
// per atom, lane n owning the 24 harmonic accumulators A_nlm and B_nlm of
// radial function n. Spin-carrying atoms occupy the leading index range and
// every grid is split so that a wavefront never mixes species; neighbour
// rows list spin carriers first, so the pair type tau, and with it every
// coefficient address, is uniform across the wavefront inside each loop.
// Sums over neighbours run in list order (ascending atom index): results are
// deterministic and independent of how replicas are batched.
//
// Gather without atomics: the backward pass writes, per listed pair (i,j),
// dE_i/dd_ij and dE_i/ds_j into a pair record; a gather kernel then forms
// F_k = sum_j dE_k/dd_kj - sum_j dE_j/dd_jk and H_k = -(dE_k/ds_k + sum_j dE_j/ds_k)
// by reading the partner's record at the reverse slot.
#include "engine.h"

namespace nep {

namespace {

// grid split: blocks [0, nbFe) take spin carriers, the rest the others
__device__ inline int atom_of_block(const Sys &S, int per_block, int nbFe, int local, bool &fe) {
    const int b = blockIdx.x;
    if (b < nbFe) {
        fe = true;
        const int i = b * per_block + local;
        return i < S.N_fe ? i : -1;
    }
    fe = false;
    const int i = S.N_fe + (b - nbFe) * per_block + local;
    return i < S.N ? i : -1;
}

// i, or -1 when its replica is not advancing (paused for a new colouring,
// finished, or its step void): the force-field kernels leave such atoms alone
__device__ inline int live(const Sys &S, int i) { return i >= 0 && S.rep[S.rid[i]].active ? i : -1; }

template <typename real>
__device__ inline void load_spin(const d4 *sp, int j, real s[3]) {
    const d4 v = sp[j];
    s[0] = (real)v.x;
    s[1] = (real)v.y;
    s[2] = (real)v.z;
}

// displacement to an already loaded neighbour position, in FP64, then cast
template <typename real>
__device__ inline real geom_p(const Img &R, const d4 &pi, const d4 &pj, real d[3]) {
    double dx, dy, dz;
    min_image(R, pi, pj, dx, dy, dz);
    d[0] = (real)dx;
    d[1] = (real)dy;
    d[2] = (real)dz;
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// C[k] = sum_n Fp[n] c[n][k]  (coefficients wave-uniform)
template <typename real>
__device__ inline void contract(const real *c, const real *Fp, int nn, real C[NB]) {
#pragma unroll
    for (int k = 0; k < NB; k++) C[k] = 0;
    // once per atom: rolled, so the coefficients are loaded nine at a time
#pragma unroll 1
    for (int n = 0; n < nn; n++) {
        const real f = Fp[n];
#pragma unroll
        for (int k = 0; k < NB; k++) C[k] += f * c[n * NB + k];
    }
}

// The same, with the atom's NR values read in one burst and the loop
// unrolled: for the per-atom coefficient kernels, whose many resident waves
// would otherwise evict an atom's row between the rolled loop's reads of it.
template <typename real>
__device__ inline void contract_burst(const real *c, const real *Fp, real C[NB]) {
    real f[NR];
#pragma unroll
    for (int n = 0; n < NR; n++) f[n] = Fp[n];
#pragma unroll
    for (int k = 0; k < NB; k++) C[k] = 0;
#pragma unroll
    for (int n = 0; n < NR; n++)
#pragma unroll
        for (int k = 0; k < NB; k++) C[k] += f[n] * c[n * NB + k];
}

template <typename real>
__device__ inline real dotk(const real C[NB], const real f[NB]) {
    real s = 0;
#pragma unroll
    for (int k = 0; k < NB; k++) s += C[k] * f[k];
    return s;
}

template <typename real>
__device__ inline real xor_sum8(real v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    return v;
}

// -------------------------------------------------------------------------
// forward: radial set (lane per atom)
// -------------------------------------------------------------------------

template <typename real>
__global__ void __launch_bounds__(256) k_desc_radial(Sys S, const real *__restrict__ C, Work<real> W,
                                                     const d4 *spin, int nbFe) {
    bool fe;
    const int i = live(S, atom_of_block(S, 256, nbFe, threadIdx.x, fe));
    if (i < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_R, rc2 = rc * rc;
    const int cnt = S.cntR[i], nfe = S.cntFeR[i];
    const size_t ld = S.N;
    real *q = W.q + (size_t)i * DP;
    real qR[NR], qE[NR], qD[NR], qA[NR], qS[NR];
#pragma unroll
    for (int n = 0; n < NR; n++) qR[n] = qE[n] = qD[n] = qA[n] = qS[n] = 0;
    real si[3];
    load_spin(spin, i, si);
    if (fe && S.mag) {
        real FR[NB], FE[NB], FD[NB], FA[NB], FS[NB];
#pragma unroll
        for (int k = 0; k < NB; k++) FR[k] = FE[k] = FD[k] = FA[k] = FS[k] = 0;
        // neighbour index two slots ahead, position and spin one slot ahead
        int j1 = 0 < nfe ? S.nbrR[i] : 0;
        int j2 = 1 < nfe ? S.nbrR[ld + i] : j1;
        d4 p1 = S.pos[j1], v1 = spin[j1];
        for (int s = 0; s < nfe; s++) {
            const d4 pj = p1, vj = v1;
            j1 = j2;
            p1 = S.pos[j1];
            v1 = spin[j1];
            if (s + 2 < nfe) j2 = S.nbrR[(size_t)(s + 2) * ld + i];
            real d[3];
            const real r2 = geom_p(R, pi, pj, d);
            if (r2 >= rc2) continue;
            real r, ir;
            r_and_inv(r2, r, ir);
            const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
            real f[NB];
            radial_basis(r, rc, f);
            const real sj[3] = {(real)vj.x, (real)vj.y, (real)vj.z};
            const real ss = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
            const real cx = si[1] * sj[2] - si[2] * sj[1], cy = si[2] * sj[0] - si[0] * sj[2],
                       cz = si[0] * sj[1] - si[1] * sj[0];
            const real dm = rh[0] * cx + rh[1] * cy + rh[2] * cz;
            const real a = si[0] * rh[0] + si[1] * rh[1] + si[2] * rh[2];
            const real b = sj[0] * rh[0] + sj[1] * rh[1] + sj[2] * rh[2];
            const real ab = a * b, aa = a * a;
#pragma unroll
            for (int k = 0; k < NB; k++) {
                FR[k] += f[k];
                FE[k] += f[k] * ss;
                FD[k] += f[k] * dm;
                FA[k] += f[k] * ab;
                FS[k] += f[k] * aa;
            }
        }
        // contract with tau = (Fe, Fe) coefficients
        for (int n = 0; n < NR; n++) {
            const int o = (0 * NR + n) * NB;
            real r_ = 0, e_ = 0, d_ = 0, a_ = 0, s_ = 0;
#pragma unroll
            for (int k = 0; k < NB; k++) {
                r_ += (C + P_CR)[o + k] * FR[k];
                e_ += (C + P_CEX)[o + k] * FE[k];
                d_ += (C + P_CDM)[o + k] * FD[k];
                a_ += (C + P_CAN)[o + k] * FA[k];
                s_ += (C + P_CSI)[o + k] * FS[k];
            }
            qR[n] = r_;
            qE[n] = e_;
            qD[n] = d_;
            qA[n] = a_;
            qS[n] = s_;
        }
        // non-magnetic neighbours: only the radial and single-ion channels survive
#pragma unroll
        for (int k = 0; k < NB; k++) FR[k] = FS[k] = 0;
        int j1_ = nfe < cnt ? S.nbrR[(size_t)(nfe) * ld + i] : 0;
        int j2_ = nfe + 1 < cnt ? S.nbrR[(size_t)(nfe + 1) * ld + i] : j1_;
        d4 p1_ = S.pos[j1_];
        for (int s = nfe; s < cnt; s++) {
            const int j = j1_;
            const d4 pj_ = p1_;
            j1_ = j2_;
            p1_ = S.pos[j1_];
            if (s + 2 < cnt) j2_ = S.nbrR[(size_t)(s + 2) * ld + i];
            real d[3];
            const real r2 = geom_p(R, pi, pj_, d);
            if (r2 >= rc2) continue;
            real r, ir;
            r_and_inv(r2, r, ir);
            real f[NB];
            radial_basis(r, rc, f);
            const real a = (si[0] * d[0] + si[1] * d[1] + si[2] * d[2]) * ir;
            const real aa = a * a;
#pragma unroll
            for (int k = 0; k < NB; k++) {
                FR[k] += f[k];
                FS[k] += f[k] * aa;
            }
        }
        for (int n = 0; n < NR; n++) {
            const int o = (1 * NR + n) * NB;
            real r_ = 0, s_ = 0;
#pragma unroll
            for (int k = 0; k < NB; k++) {
                r_ += (C + P_CR)[o + k] * FR[k];
                s_ += (C + P_CSI)[o + k] * FS[k];
            }
            qR[n] += r_;
            qS[n] += s_;
        }
        q[D_OS] = si[0] * si[0] + si[1] * si[1] + si[2] * si[2];
    } else {
        for (int part = 0; part < 2; part++) {
            real FR[NB];
#pragma unroll
            for (int k = 0; k < NB; k++) FR[k] = 0;
            const int b = part ? nfe : 0, e = part ? cnt : nfe;
            int j1_ = b < e ? S.nbrR[(size_t)(b) * ld + i] : 0;
            int j2_ = b + 1 < e ? S.nbrR[(size_t)(b + 1) * ld + i] : j1_;
            d4 p1_ = S.pos[j1_];
            for (int s = b; s < e; s++) {
                const int j = j1_;
                const d4 pj_ = p1_;
                j1_ = j2_;
                p1_ = S.pos[j1_];
                if (s + 2 < e) j2_ = S.nbrR[(size_t)(s + 2) * ld + i];
                real d[3];
                const real r2 = geom_p(R, pi, pj_, d);
                if (r2 >= rc2) continue;
                real f[NB], r, ir;
                r_and_inv(r2, r, ir);
                radial_basis(r, rc, f);
#pragma unroll
                for (int k = 0; k < NB; k++) FR[k] += f[k];
            }
            const int tau = (fe ? 0 : 2) + part;
            for (int n = 0; n < NR; n++) {
                const int o = (tau * NR + n) * NB;
                real r_ = 0;
#pragma unroll
                for (int k = 0; k < NB; k++) r_ += (C + P_CR)[o + k] * FR[k];
                qR[n] += r_;
            }
        }
        q[D_OS] = 0;
    }
#pragma unroll
    for (int n = 0; n < NR; n++) {
        q[D_R + n] = qR[n];
        q[D_EX + n] = qE[n];
    }
    // The structural-only read-out contracts over the first 40 entries (the
    // zero onsite and exchange entries 37-39 included): it never reads the
    // later magnetic channels, which stay unwritten there.
    if (S.mag) {
#pragma unroll
        for (int n = 0; n < NR; n++) {
            q[D_DM + n] = qD[n];
            q[D_AN + n] = qA[n];
            q[D_SI + n] = qS[n];
        }
    }
}

// -------------------------------------------------------------------------
// angular-set kernels: one wavefront = 8 atoms x 8 lanes
// Every neighbour loop runs in two phases, spin-carrying neighbours first
// (they lead each list) and then the others, so within a phase the pair type
// tau and thus every coefficient address is uniform across the wavefront and
// the coefficients are scalar operands.
// -------------------------------------------------------------------------

constexpr int ANG_ATOMS = 8;             // atoms per workgroup
constexpr int ANG_TW = 2 * NA + NLM;     // staged values per neighbour
constexpr int ANG_TS = 8 * ANG_TW + 1;   // per-atom stride (shifts LDS banks)

template <typename real>
__device__ inline real dotc(const real *c, const real f[NB]) {
    real s = 0;
#pragma unroll
    for (int k = 0; k < NB; k++) s += c[k] * f[k];
    return s;
}

// forward: per round, lanes stage eight neighbours of their atom (radial
// functions g^A_n and (s_i.s_j) g^sa_n for all n, the 24 harmonics) in LDS,
// then lane n accumulates A_nlm and B_nlm over the staged neighbours. B only
// has spin-carrying pairs (spin-carrying centre, first phase).
// Pass modes: PASS_FULL stores A (all atoms) and B (spin carriers) for the
// backward pass; PASS_SPIN (spin carriers only) stores A for the coupling
// assembly; PASS_SPIN_REUSE (same positions as the preceding PASS_SPIN)
// takes A from it and only recomputes B and q^sa.
template <typename real>
__global__ void __launch_bounds__(64) k_desc_angular(Sys S, const real *__restrict__ C, Work<real> W,
                                                     const d4 *spin, int nbFe, int mode) {
    __shared__ real tile[ANG_ATOMS * ANG_TS];
    __shared__ int smax[2];
    const int lane = threadIdx.x & 7, slot = threadIdx.x >> 3;
    bool fe;
    const int i = live(S, atom_of_block(S, ANG_ATOMS, nbFe, slot, fe));
    const bool reuse = mode == PASS_SPIN_REUSE;
    if (threadIdx.x == 0) smax[0] = smax[1] = 0;
    __syncthreads();
    int cnt = 0, nfe = 0;
    d4 pi = {0, 0, 0, 0};
    real si[3] = {0, 0, 0};
    Img R = {};
    if (i >= 0) {
        cnt = S.cntA[i];
        nfe = S.cntFeA[i];
        pi = S.pos[i];
        load_spin(spin, i, si);
        R = img_of(S.rep[S.rid[i]]);
        if (lane == 0) {
            atomicMax(&smax[0], nfe);
            atomicMax(&smax[1], cnt - nfe);
        }
    }
    __syncthreads();
    const int n = lane < NA ? lane : NA - 1;
    const int m0 = 3 * lane;                 // this lane's three harmonics, for every n
    const real rc = (real)RC_A, rc2 = rc * rc;
    const size_t ld = S.N;
    real A[NA][3], B[NA][3];
#pragma unroll
    for (int x = 0; x < NA; x++)
#pragma unroll
        for (int m = 0; m < 3; m++) A[x][m] = B[x][m] = 0;
    real *my = tile + slot * ANG_TS;
    const int nparts = reuse ? 1 : 2;
    for (int part = 0; part < nparts; part++) {
        const int tau = (fe ? 0 : 2) + part;
        const real *cA = C + P_CA + tau * NA * NB, *cS = C + P_CSA + tau * NA * NB;
        const bool spins = S.mag && fe && part == 0;
        const int b = part ? nfe : 0, e = part ? cnt : nfe;
        const int rounds = (smax[part] + 7) >> 3;
        // this lane's neighbour index two rounds ahead, position and spin one round ahead
        const int s0 = b + lane;
        int jc = s0 < e ? S.nbrA[(size_t)s0 * ld + i] : 0;
        int jn = s0 + 8 < e ? S.nbrA[(size_t)(s0 + 8) * ld + i] : jc;
        d4 pc = S.pos[jc], vc = {0, 0, 0, 0};
        if (spins) vc = spin[jc];
        for (int rd = 0; rd < rounds; rd++) {
            const int s = b + rd * 8 + lane;
            const d4 pj = pc, vj = vc;
            jc = jn;
            pc = S.pos[jc];
            if (spins) vc = spin[jc];
            if (s + 16 < e) jn = S.nbrA[(size_t)(s + 16) * ld + i];
            real *en = my + lane * ANG_TW;
            if (s < e) {
                real d[3];
                const real r2 = geom_p(R, pi, pj, d);
                if (r2 < rc2) {
                    real r, ir;
                    r_and_inv(r2, r, ir);
                    real f[NB];
                    radial_basis(r, rc, f);
                    if (spins) {
                        const real sj[3] = {(real)vj.x, (real)vj.y, (real)vj.z};
                        const real sig = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
#pragma unroll
                        for (int nn = 0; nn < NA; nn++) en[NA + nn] = sig * dotc(cS + nn * NB, f);
                    }
                    if (!reuse) {
#pragma unroll
                        for (int nn = 0; nn < NA; nn++) en[nn] = dotc(cA + nn * NB, f);
                    }
                    real Y[NLM];
                    harmonics(d[0] * ir, d[1] * ir, d[2] * ir, Y);
#pragma unroll
                    for (int m = 0; m < NLM; m++) en[2 * NA + m] = Y[m];
                } else {
#pragma unroll
                    for (int k = 0; k < ANG_TW; k++) en[k] = 0;
                }
            }
            __syncthreads();
            const int qn = min(8, e - (b + rd * 8));
            if (spins && !reuse) {
                for (int q = 0; q < qn; q++) {
                    const real *e2 = my + q * ANG_TW;
                    const real y0 = e2[2 * NA + m0], y1 = e2[2 * NA + m0 + 1], y2 = e2[2 * NA + m0 + 2];
#pragma unroll
                    for (int x = 0; x < NA; x++) {
                        const real ga = e2[x], gs = e2[NA + x];
                        A[x][0] += ga * y0;
                        A[x][1] += ga * y1;
                        A[x][2] += ga * y2;
                        B[x][0] += gs * y0;
                        B[x][1] += gs * y1;
                        B[x][2] += gs * y2;
                    }
                }
            } else if (spins) {
                for (int q = 0; q < qn; q++) {
                    const real *e2 = my + q * ANG_TW;
                    const real y0 = e2[2 * NA + m0], y1 = e2[2 * NA + m0 + 1], y2 = e2[2 * NA + m0 + 2];
#pragma unroll
                    for (int x = 0; x < NA; x++) {
                        const real gs = e2[NA + x];
                        B[x][0] += gs * y0;
                        B[x][1] += gs * y1;
                        B[x][2] += gs * y2;
                    }
                }
            } else {
                for (int q = 0; q < qn; q++) {
                    const real *e2 = my + q * ANG_TW;
                    const real y0 = e2[2 * NA + m0], y1 = e2[2 * NA + m0 + 1], y2 = e2[2 * NA + m0 + 2];
#pragma unroll
                    for (int x = 0; x < NA; x++) {
                        const real ga = e2[x];
                        A[x][0] += ga * y0;
                        A[x][1] += ga * y1;
                        A[x][2] += ga * y2;
                    }
                }
            }
            __syncthreads();
        }
    }
    // regroup through LDS: lane n takes A_n and B_n over all 24 harmonics
    real An[NLM], Bn[NLM];
    if (!reuse) {
#pragma unroll
        for (int x = 0; x < NA; x++)
#pragma unroll
            for (int m = 0; m < 3; m++) my[x * NLM + m0 + m] = A[x][m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NLM; m++) An[m] = my[n * NLM + m];
        __syncthreads();
    }
    if (fe && S.mag) {
#pragma unroll
        for (int x = 0; x < NA; x++)
#pragma unroll
            for (int m = 0; m < 3; m++) my[x * NLM + m0 + m] = B[x][m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NLM; m++) Bn[m] = my[n * NLM + m];
    } else {
#pragma unroll
        for (int m = 0; m < NLM; m++) Bn[m] = 0;
    }
    if (i < 0 || lane >= NA) return;
    real *ab = W.AB + ((size_t)i * NA + n) * NAB;
    real *q = W.q + (size_t)i * DP;
    if (reuse) {
#pragma unroll
        for (int m = 0; m < NLM; m++) An[m] = ab[m];
    }
    real qa[4] = {0, 0, 0, 0}, qs[4] = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < NLM; m++) {
        qa[l_of_lm(m) - 1] += An[m] * An[m];
        qs[l_of_lm(m) - 1] += An[m] * Bn[m];
    }
#pragma unroll
    for (int l = 0; l < 4; l++) {
        if (!reuse) q[D_A + 4 * n + l] = qa[l];
        if (S.mag) q[D_SA + 4 * n + l] = qs[l];   // beyond the structural-only read-out's entries
    }
    if (!reuse) {
#pragma unroll
        for (int m = 0; m < NLM; m++) ab[m] = An[m];
    }
    if (fe && S.mag && mode == PASS_FULL) {   // B only for the spin-carrying backward
#pragma unroll
        for (int m = 0; m < NLM; m++) ab[NLM + m] = Bn[m];
    }
}

// -------------------------------------------------------------------------
// per-species read-out on the matrix cores
//   Z = Q W0^T + b0 (atoms x 64), E_i = b1 + w1 . tanh(Z_i),
//   Fp = [(1 - tanh^2(Z)) * w1] W0 (atoms x 104)
// One wavefront takes a tile of 16 atoms of one species; W0^T of that species
// is staged in LDS once per workgroup. Operand layout of v_mfma_*_16x16x4:
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k. Accumulator element r of
// lane l holds column l % 16 and row 4 (l / 16) + r for the FP32
// instruction, row (l / 16) + 4 r for the FP64 one (checked on gfx950).
// -------------------------------------------------------------------------

template <typename real>
struct MF;
template <>
struct MF<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    __device__ static acc_t mma(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct MF<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int kq, int r) { return 4 * kq + r; }
};

constexpr int MLP_WAVES = 8;           // 8 wavefronts x 16 atoms per workgroup
constexpr int MLP_ATOMS = 16 * MLP_WAVES;
// LDS row strides of W0^T and of the per-wave hidden tile. The MFMA operand
// reads walk 16 rows (lanes i16) and 4 columns (lanes kq); a stride of 2
// dwords mod 64 for 8-byte and 4 dwords mod 64 for 4-byte elements puts those
// 64 reads on distinct banks.
template <typename real>
struct MlpLds;
template <>
struct MlpLds<double> {
    static constexpr int LD = NH + 1;
};
template <>
struct MlpLds<float> {
    static constexpr int LD = NH + 4;
};

// KD: descriptor entries the read-out contracts over (104 for the spin-aware
// model, 40 for the structural-only one, whose 37 entries lead each row)
template <typename real, int KD>
__global__ void __launch_bounds__(512) k_mlp(Sys S, ModelDev<real> M, Work<real> W, int nbFe) {
    typedef typename MF<real>::acc_t acc_t;
    constexpr int WLD = MlpLds<real>::LD, GLD = MlpLds<real>::LD;
    constexpr bool f64 = sizeof(real) == 8;
    constexpr int KDT = (KD + 15) / 16 * 16, NT = KDT / 16;
    __shared__ real sW[KDT * WLD];
    __shared__ real sG[f64 ? 1 : MLP_WAVES * 16 * GLD];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool fe = (int)blockIdx.x < nbFe;
    const int t = fe ? 0 : 1;
    const int end = fe ? S.N_fe : S.N;
    const int a0 = (fe ? blockIdx.x * MLP_ATOMS : S.N_fe + (blockIdx.x - nbFe) * MLP_ATOMS) + wave * 16;
    const real *W0 = M.W0 + (size_t)t * DP * NH;
    for (int x = threadIdx.x; x < KDT * NH; x += blockDim.x) {
        const int d = x / NH, h = x - d * NH;
        sW[d * WLD + h] = d < KD ? W0[d * NH + h] : real(0);
    }
    __syncthreads();
    const int i16 = lane & 15, kq = lane >> 4;
    const int arow = a0 + i16;
    const bool rv = arow < end && live(S, arow) >= 0;
    const real *qrow = W.q + (size_t)(rv ? arow : 0) * DP;
    if constexpr (f64) {
        // Transposed form: Z^T = W0 Q^T + b0 (hidden x atoms). With the FP64
        // accumulator layout, element r of tile mt in lane l is Z^T[16 mt +
        // l/16 + 4 r][l % 16], which is exactly the B operand lane l supplies
        // for k-step ks = 4 mt + r of Fp^T = W0^T G^T: no transposition.
        real qa[KD / 4];
#pragma unroll
        for (int ks = 0; ks < KD / 4; ks++) qa[ks] = rv ? qrow[ks * 4 + kq] : real(0);
        acc_t z[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int r = 0; r < 4; r++) z[mt][r] = M.b0[t * NH + 16 * mt + kq + 4 * r];
#pragma unroll
        for (int ks = 0; ks < KD / 4; ks++) {
#pragma unroll
            for (int mt = 0; mt < 4; mt++)
                z[mt] = MF<real>::mma(sW[(ks * 4 + kq) * WLD + mt * 16 + i16], qa[ks], z[mt]);
        }
        real e = 0;
        acc_t g[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int hh = 16 * mt + kq + 4 * r;
                const real w = M.w1[t * NH + hh];
                const real a = dtanh<real>(z[mt][r]);
                e += w * a;
                g[mt][r] = w * (real(1) - a * a);
            }
        e += __shfl_xor(e, 16);
        e += __shfl_xor(e, 32);
        if (kq == 0 && rv) W.Ei[arow] = M.b1[t] + e;
        // Fp^T = W0^T G^T: A = W0^T tile from LDS, B = this lane's g; the
        // descriptor tiles in passes of at most four to bound the registers
        real *fp = W.Fp + (size_t)(rv ? arow : 0) * DP;
#pragma unroll
        for (int half = 0; half < 2; half++) {
            constexpr int H0 = 4;
            const int d0 = half ? H0 : 0, nd = half ? NT - H0 : (NT < H0 ? NT : H0);
            if (nd <= 0) continue;
            acc_t f[H0];
#pragma unroll
            for (int x = 0; x < H0; x++) f[x] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < NH / 4; ks++) {
#pragma unroll
                for (int x = 0; x < H0; x++)
                    if (x < nd)
                        f[x] = MF<real>::mma(sW[((d0 + x) * 16 + i16) * WLD + ks * 4 + kq], g[ks >> 2][ks & 3], f[x]);
            }
            if (rv) {
#pragma unroll
                for (int x = 0; x < H0; x++)
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int d = (d0 + x) * 16 + kq + 4 * r;
                        if (x < nd && d < KD) fp[d] = f[x][r];
                    }
            }
        }
        return;
    }
    acc_t acc[4];
#pragma unroll
    for (int jt = 0; jt < 4; jt++) {
        const real b0 = M.b0[t * NH + jt * 16 + i16];
        acc[jt] = acc_t{b0, b0, b0, b0};
    }
    {
        // this lane's 26 descriptor values, all loads in flight at once
        real qa[KD / 4];
#pragma unroll
        for (int ks = 0; ks < KD / 4; ks++) qa[ks] = rv ? qrow[ks * 4 + kq] : real(0);
#pragma unroll
        for (int ks = 0; ks < KD / 4; ks++) {
#pragma unroll
            for (int jt = 0; jt < 4; jt++)
                acc[jt] = MF<real>::mma(qa[ks], sW[(ks * 4 + kq) * WLD + jt * 16 + i16], acc[jt]);
        }
    }
    // activation, energy and the hidden-layer gradient
    real e[4] = {0, 0, 0, 0};
    real *g = sG + wave * 16 * GLD;
#pragma unroll
    for (int jt = 0; jt < 4; jt++) {
        const real w = M.w1[t * NH + jt * 16 + i16];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const real a = dtanh<real>(acc[jt][r]);
            e[r] += w * a;
            g[MF<real>::row(kq, r) * GLD + jt * 16 + i16] = w * (real(1) - a * a);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) e[r] += __shfl_xor(e[r], m);
    }
    if (i16 == 0) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = a0 + MF<real>::row(kq, r);
            if (row < end && live(S, row) >= 0) W.Ei[row] = M.b1[t] + e[r];
        }
    }
    __syncthreads();
    // Fp = G W0: A[i][k] = G[i][k], B[k][j] = W0[k][j] = sW[j][k]
    acc_t f[NT];
#pragma unroll
    for (int jt = 0; jt < NT; jt++) f[jt] = acc_t{0, 0, 0, 0};
    for (int ks = 0; ks < NH / 4; ks++) {
        const real a = g[i16 * GLD + ks * 4 + kq];
#pragma unroll
        for (int jt = 0; jt < NT; jt++) f[jt] = MF<real>::mma(a, sW[(jt * 16 + i16) * WLD + ks * 4 + kq], f[jt]);
    }
#pragma unroll
    for (int jt = 0; jt < NT; jt++) {
        const int col = jt * 16 + i16;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = a0 + MF<real>::row(kq, r);
            if (row < end && col < KD && live(S, row) >= 0) W.Fp[(size_t)row * DP + col] = f[jt][r];
        }
    }
}

// -------------------------------------------------------------------------
// backward: radial set (lane per atom)
// -------------------------------------------------------------------------

template <typename real>
__device__ inline void put_pair(real *pb, size_t idx, const real G[3], const real h[3]) {
    real *p = pb + idx * 6;
    p[0] = G[0];
    p[1] = G[1];
    p[2] = G[2];
    p[3] = h[0];
    p[4] = h[1];
    p[5] = h[2];
}

// Per atom i of species t, its radial-set coefficients contracted with its
// own Fp, for each neighbour species p: CR_p[k] = sum_n c^R_{2t+p}[n][k] Fp^R_n
// and, on spin carriers, CS_p[k] = sum_n c^si_{2t+p}[n][k] Fp^si_n (zero on
// the others). Stored as [CR_0 | CR_1 | CS_0 | CS_1][N][NB]: a neighbour reads
// the NB values of its own species (and NB more if it carries a spin), and
// atoms adjacent in memory share cache lines. Spin carriers also get the exchange, DMI and
// anisotropic-exchange coefficients (Fe-Fe pairs), [N_fe][CE, CD, CA].
template <typename real>
__device__ inline void mag_coef(const real *__restrict__ C, const real *Fp, real *m) {
    real CX[NB];
    contract_burst((C + P_CEX), Fp + D_EX, CX);
#pragma unroll
    for (int k = 0; k < NB; k++) m[k] = CX[k];
    contract_burst((C + P_CDM), Fp + D_DM, CX);
#pragma unroll
    for (int k = 0; k < NB; k++) m[NB + k] = CX[k];
    contract_burst((C + P_CAN), Fp + D_AN, CX);
#pragma unroll
    for (int k = 0; k < NB; k++) m[2 * NB + k] = CX[k];
}

template <typename real>
__global__ void __launch_bounds__(256) k_radial_coef(Sys S, const real *__restrict__ C, Work<real> W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N || live(S, i) < 0) return;
    const bool fe = i < S.N_fe;
    const int t = fe ? 0 : 1;
    const real *Fp = W.Fp + (size_t)i * DP;
    const size_t ld = S.N;
#pragma unroll 1
    for (int p = 0; p < 2; p++) {
        real CR[NB];
        contract_burst((C + P_CR) + (2 * t + p) * NR * NB, Fp + D_R, CR);
        real *oR = W.rcoef + ((size_t)p * ld + i) * NB;
#pragma unroll
        for (int k = 0; k < NB; k++) oR[k] = CR[k];
        if (fe && S.mag) {   // single-ion block, read only for spin-carrying partners
            real CS[NB];
            contract_burst((C + P_CSI) + p * NR * NB, Fp + D_SI, CS);
            real *oS = W.rcoef + ((size_t)(2 + p) * ld + i) * NB;
#pragma unroll
            for (int k = 0; k < NB; k++) oS[k] = CS[k];
        }
    }
    if (fe && S.mag) mag_coef(C, Fp, W.mcoef + (size_t)i * MCOEF);
}

// the exchange, DMI and anisotropic-exchange coefficients alone, spin carriers
// (the spin-step passes)
template <typename real>
__global__ void __launch_bounds__(256) k_mag_coef(Sys S, const real *__restrict__ C, Work<real> W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe || live(S, i) < 0) return;
    mag_coef(C, W.Fp + (size_t)i * DP, W.mcoef + (size_t)i * MCOEF);
}

// Structural part of the radial-set backward pass: the radial channel of
// every pair and the single-ion term of spin-carrying centres, lane per atom.
// Both halves of each pair come from this lane: G_ij = dE_i/dd_ij from the
// atom's own coefficients and G_ji = dE_j/dd_ji from the neighbour's
// contracted block (and its spin), so F_i = sum_j (G_ij - G_ji) needs no
// pair records. Own sums: F_i and dE_i/ds_i (single-ion and onsite).
template <typename real>
__device__ inline void partner_radial(const real *cR, const real *cS, bool fe_j, const d4 *spin, int j, real r,
                                      real ir, const real rh[3], const real f[NB], const real df[NB], real Gj[3]) {
    const real dgR = dotc(cR + (size_t)j * NB, df);
    if (fe_j) {
        real sj[3];
        load_spin(spin, j, sj);
        const real gS = dotc(cS + (size_t)j * NB, f), dgS = dotc(cS + (size_t)j * NB, df);
        // rhat_ji = -rhat_ij
        const real a = -(sj[0] * rh[0] + sj[1] * rh[1] + sj[2] * rh[2]);
        const real radial = dgR + dgS * a * a;
        const real ks = real(2) * gS * a * ir;
#pragma unroll
        for (int x = 0; x < 3; x++) Gj[x] = -radial * rh[x] + ks * (sj[x] + a * rh[x]);
    } else {
#pragma unroll
        for (int x = 0; x < 3; x++) Gj[x] = -dgR * rh[x];
    }
}

// Optional short-range repulsion of one pair of type tau at distance r: the
// universal screened-Coulomb (ZBL) potential K Z_i Z_j / r phi(r/a), phi a
// sum of four exponentials of r/a, times the switch
// (1 + cos(pi (r - r_inner)/(r_outer - r_inner)))/2 above r_inner. Z is the
// model's short-range block (products K Z_i Z_j, inverse screening lengths,
// r_inner, r_outer, pi/(r_outer - r_inner)). V and dV/dr of the pair.
template <typename real>
__device__ inline void short_range(const real *Z, int tau, real r, real ir, real &V, real &dV) {
    const real ia = Z[4 + tau];
    const real c0 = real(0.18175) * dexp<real>(real(-3.19980) * ia * r);
    const real c1 = real(0.50986) * dexp<real>(real(-0.94229) * ia * r);
    const real c2 = real(0.28022) * dexp<real>(real(-0.40290) * ia * r);
    const real c3 = real(0.02817) * dexp<real>(real(-0.20162) * ia * r);
    const real phi = c0 + c1 + c2 + c3;
    const real dphi = -ia * (real(3.19980) * c0 + real(0.94229) * c1 + real(0.40290) * c2 + real(0.20162) * c3);
    const real v = Z[tau] * phi * ir;
    const real dv = Z[tau] * (dphi - phi * ir) * ir;
    real s = 1, ds = 0;
    if (r > Z[8]) {
        const real w = Z[10], x = w * (r - Z[8]);
        s = real(0.5) * (real(1) + dcos<real>(x));
        ds = real(-0.5) * w * dsin<real>(x);
    }
    V = v * s;
    dV = dv * s + v * ds;
}

template <typename real>
__global__ void __launch_bounds__(256) k_bwd_radial(Sys S, const real *__restrict__ C, Work<real> W, int nbFe) {
    bool fe;
    const int i = live(S, atom_of_block(S, 256, nbFe, threadIdx.x, fe));
    if (i < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_R, rc2 = rc * rc;
    const int cnt = S.cntR[i], nfe = S.cntFeR[i];
    const size_t ld = S.N;
    const real *Fp = W.Fp + (size_t)i * DP;
    // the neighbours' contracted blocks for this atom's species
    const real *nR = W.rcoef + (size_t)(fe ? 0 : 1) * ld * NB, *nS = W.rcoef + (size_t)(fe ? 2 : 3) * ld * NB;
    real F[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    // short-range term: half of every pair's energy goes to E_i; the force of
    // the pair on i is V'(r) rhat_ij (both halves)
    const real *Z = C + M_ZBL;
    const bool zon = Z[11] != real(0);
    const real zr2 = zon ? Z[9] : real(0);
    real esr = 0;
    if (fe && S.mag) {
        real si[3];
        load_spin(S.spin, i, si);
        const real os2 = real(2) * Fp[D_OS];
        h[0] = os2 * si[0];
        h[1] = os2 * si[1];
        h[2] = os2 * si[2];
        // onsite moment-length term a|s|^2 + b|s|^4: its energy and dE/ds
        const RepDev &Rr = S.rep[S.rid[i]];
        if (Rr.landau_a != 0.0 || Rr.landau_b != 0.0) {
            const real la = (real)Rr.landau_a, lb = (real)Rr.landau_b;
            const real s2 = si[0] * si[0] + si[1] * si[1] + si[2] * si[2];
            const real kl = real(2) * la + real(4) * lb * s2;
            h[0] += kl * si[0];
            h[1] += kl * si[1];
            h[2] += kl * si[2];
            esr += la * s2 + lb * s2 * s2;
        }
        for (int part = 0; part < 2; part++) {
            real CR[NB], CS[NB];
            contract((C + P_CR) + part * NR * NB, Fp + D_R, NR, CR);
            contract((C + P_CSI) + part * NR * NB, Fp + D_SI, NR, CS);
            const int b = part ? nfe : 0, e = part ? cnt : nfe;
            int j1_ = b < e ? S.nbrR[(size_t)(b) * ld + i] : 0;
            int j2_ = b + 1 < e ? S.nbrR[(size_t)(b + 1) * ld + i] : j1_;
            d4 p1_ = S.pos[j1_];
            for (int s = b; s < e; s++) {
                const int j = j1_;
                const d4 pj_ = p1_;
                j1_ = j2_;
                p1_ = S.pos[j1_];
                if (s + 2 < e) j2_ = S.nbrR[(size_t)(s + 2) * ld + i];
                real d[3];
                const real r2 = geom_p(R, pi, pj_, d);
                if (r2 >= rc2) continue;
                real r, ir;
                r_and_inv(r2, r, ir);
                const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
                real f[NB], df[NB];
                radial_basis_d(r, rc, f, df);
                const real dgR = dotk(CR, df);
                const real gS = dotk(CS, f), dgS = dotk(CS, df);
                const real a = si[0] * rh[0] + si[1] * rh[1] + si[2] * rh[2];
                const real radial = dgR + dgS * a * a;
                const real ks = real(2) * gS * a * ir;
                real Gj[3];
                partner_radial(nR, nS, S.mag && part == 0, S.spin, j, r, ir, rh, f, df, Gj);
#pragma unroll
                for (int x = 0; x < 3; x++) {
                    const real G = radial * rh[x] + ks * (si[x] - a * rh[x]);
                    h[x] += real(2) * gS * a * rh[x];
                    F[x] += G - Gj[x];
                }
                if (r < zr2) {
                    real V, dV;
                    short_range(Z, part, r, ir, V, dV);
                    esr += real(0.5) * V;
#pragma unroll
                    for (int x = 0; x < 3; x++) F[x] += dV * rh[x];
                }
            }
        }
    } else {
        for (int part = 0; part < 2; part++) {
            real CR[NB];
            contract((C + P_CR) + ((fe ? 0 : 2) + part) * NR * NB, Fp + D_R, NR, CR);
            const int b = part ? nfe : 0, e = part ? cnt : nfe;
            int j1_ = b < e ? S.nbrR[(size_t)(b) * ld + i] : 0;
            int j2_ = b + 1 < e ? S.nbrR[(size_t)(b + 1) * ld + i] : j1_;
            d4 p1_ = S.pos[j1_];
            for (int s = b; s < e; s++) {
                const int j = j1_;
                const d4 pj_ = p1_;
                j1_ = j2_;
                p1_ = S.pos[j1_];
                if (s + 2 < e) j2_ = S.nbrR[(size_t)(s + 2) * ld + i];
                real d[3];
                const real r2 = geom_p(R, pi, pj_, d);
                if (r2 >= rc2) continue;
                real r, ir;
                r_and_inv(r2, r, ir);
                const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
                real f[NB], df[NB];
                radial_basis_d(r, rc, f, df);
                const real g = dotk(CR, df);
                real Gj[3];
                partner_radial(nR, nS, S.mag && part == 0, S.spin, j, r, ir, rh, f, df, Gj);
#pragma unroll
                for (int x = 0; x < 3; x++) F[x] += g * rh[x] - Gj[x];
                if (r < zr2) {
                    real V, dV;
                    short_range(Z, (fe ? 0 : 2) + part, r, ir, V, dV);
                    esr += real(0.5) * V;
#pragma unroll
                    for (int x = 0; x < 3; x++) F[x] += dV * rh[x];
                }
            }
        }
    }
    put_pair(W.ownR, (size_t)i, F, h);
    if (esr != real(0)) W.Ei[i] += esr;
}

// Magnetic pair part of the radial-set backward pass: exchange, DMI and
// anisotropic exchange over the spin-carrying neighbours of spin-carrying
// centres, lane per atom. The partner's pair energy e_ji has the form of e_ij
// in terms of d_ij (r_hat_ji.(s_j x s_i) = r_hat_ij.(s_i x s_j), and likewise
// for the anisotropic product), so a pair's force on i and field on s_i are
// the formulas of e_ij with the summed coefficients C_i + C_j: no records.
// Sums: F_i and dE/ds_i of these channels.
template <typename real>
__global__ void __launch_bounds__(256) k_bwd_mag(Sys S, const real *__restrict__ C, Work<real> W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe || live(S, i) < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_R, rc2 = rc * rc;
    const int nfe = min(S.cntFeR[i], MAXFE);
    const size_t ld = S.N;
    real F[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    real si[3];
    load_spin(S.spin, i, si);
    real Ci[3 * NB];
    {
        const real *m = W.mcoef + (size_t)i * MCOEF;
#pragma unroll
        for (int k = 0; k < 3 * NB; k++) Ci[k] = m[k];
    }
    // neighbour index two slots ahead, its position and spin one slot ahead
    int j1_ = 0 < nfe ? S.nbrR[i] : 0;
    int j2_ = 1 < nfe ? S.nbrR[ld + i] : j1_;
    d4 p1_ = S.pos[j1_], v1_ = S.spin[j1_];
    for (int s = 0; s < nfe; s++) {
        const int j = j1_;
        const d4 pj_ = p1_, vj_ = v1_;
        j1_ = j2_;
        p1_ = S.pos[j1_];
        v1_ = S.spin[j1_];
        if (s + 2 < nfe) j2_ = S.nbrR[(size_t)(s + 2) * ld + i];
        real d[3];
        const real r2 = geom_p(R, pi, pj_, d);
        if (r2 >= rc2) continue;
        real r, ir;
        r_and_inv(r2, r, ir);
        const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
        real f[NB], df[NB];
        radial_basis_d(r, rc, f, df);
        const real *mj = W.mcoef + (size_t)j * MCOEF;
        real CE[NB], CD[NB], CA[NB];
#pragma unroll
        for (int k = 0; k < NB; k++) {
            CE[k] = Ci[k] + mj[k];
            CD[k] = Ci[NB + k] + mj[NB + k];
            CA[k] = Ci[2 * NB + k] + mj[2 * NB + k];
        }
        const real sj[3] = {(real)vj_.x, (real)vj_.y, (real)vj_.z};
        const real gE = dotk(CE, f), dgE = dotk(CE, df);
        const real gD = dotk(CD, f), dgD = dotk(CD, df);
        const real gA = dotk(CA, f), dgA = dotk(CA, df);
        const real ss = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
        const real c[3] = {si[1] * sj[2] - si[2] * sj[1], si[2] * sj[0] - si[0] * sj[2],
                           si[0] * sj[1] - si[1] * sj[0]};
        const real w = rh[0] * c[0] + rh[1] * c[1] + rh[2] * c[2];
        const real a = si[0] * rh[0] + si[1] * rh[1] + si[2] * rh[2];
        const real b = sj[0] * rh[0] + sj[1] * rh[1] + sj[2] * rh[2];
        const real radial = dgE * ss + dgD * w + dgA * a * b;
        const real sjxr[3] = {sj[1] * rh[2] - sj[2] * rh[1], sj[2] * rh[0] - sj[0] * rh[2],
                              sj[0] * rh[1] - sj[1] * rh[0]};
        const real kd = gD * ir, ka = gA * ir;
#pragma unroll
        for (int x = 0; x < 3; x++) {
            const real pa = si[x] - a * rh[x], pb = sj[x] - b * rh[x];
            F[x] += radial * rh[x] + kd * (c[x] - w * rh[x]) + ka * (b * pa + a * pb);
            h[x] += gE * sj[x] + gD * sjxr[x] + gA * b * rh[x];
        }
    }
    put_pair(W.ownM, (size_t)i, F, h);
}

// -------------------------------------------------------------------------
// backward: angular set
//   q^A_nl = sum_m A_nlm^2, q^sa_nl = sum_m A_nlm B_nlm with
//   A_nlm = sum_j g^A_n Y_lm(rhat_ij), B_nlm = sum_j g^sa_n (s_i.s_j) Y_lm(rhat_ij)
//   dE_i/dd_ij = sum_lm [QA_lm d(g^A Y)/dd + (s_i.s_j) QS_lm d(g^sa Y)/dd]
//   with QA_nlm = 2 Fp^A_nl A_nlm + Fp^sa_nl B_nlm, QS_nlm = Fp^sa_nl A_nlm;
//   h_ij = sum_lm Y_lm sum_n QS_nlm g^sa_n, so that dE_i/ds_j = h_ij s_i and
//   the pair adds h_ij s_j to dE_i/ds_i.
// The eight lanes of an atom take its neighbours round robin, each pair in
// full; the atom's 336 QA/QS values sit in LDS. A pair record holds
// (dE_i/dd_ij, h_ij); the gather forms every sum in slot order.
// -------------------------------------------------------------------------

// Each species runs as its own launch over atoms [first, last). Atoms without
// spin work (the second species, or every atom of a structural-only model)
// keep no QS block, so that twice as many of their workgroups fit in a CU's
// LDS.
template <bool FE>
constexpr int qstride() { return (FE ? 2 : 1) * NA * NLM + 1; }

template <typename real, bool FE>
__global__ void __launch_bounds__(64) k_bwd_angular(Sys S, const real *__restrict__ C, Work<real> W, int first,
                                                    int last) {
    constexpr int QSTRIDE = qstride<FE>();
    __shared__ real sQ[ANG_ATOMS * QSTRIDE];
    const int lane = threadIdx.x & 7, slot = threadIdx.x >> 3;
    const bool fe = first < S.N_fe;    // species 0: the pair types tau = 0, 1
    int i = first + blockIdx.x * ANG_ATOMS + slot;
    i = live(S, i < last ? i : -1);
    real *Q = sQ + slot * QSTRIDE;   // QA[n][m], then QS[n][m] on spin carriers
    if (i >= 0) {
        const real *Fp = W.Fp + (size_t)i * DP;
        for (int x = lane; x < NA * NLM; x += 8) {
            const int n = x / NLM, m = x - n * NLM, l = l_of_lm(m) - 1;
            const real *ab = W.AB + ((size_t)i * NA + n) * NAB;
            const real fa = Fp[D_A + 4 * n + l];
            if (FE) {
                const real fs = Fp[D_SA + 4 * n + l];
                Q[x] = real(2) * fa * ab[m] + fs * ab[NLM + m];
                Q[NA * NLM + x] = fs * ab[m];
            } else {
                Q[x] = real(2) * fa * ab[m];
            }
        }
    }
    __syncthreads();
    if (i < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_A, rc2 = rc * rc;
    const int cnt = S.cntA[i], nfe = S.cntFeA[i];
    const size_t ld = S.N;
    real si[3];
    load_spin(S.spin, i, si);
    real Fo[3] = {0, 0, 0}, ho[3] = {0, 0, 0};     // own-side sums of this lane's pairs
    // In-cutoff pairs go to the atom's lanes by their rank among in-cutoff
    // pairs, so that the lane partial sums (and their rounding) depend on the
    // positions only and not on which farther atoms the list happens to hold.
    const int gbase = threadIdx.x & ~7;
    int rank = 0;
#pragma unroll 1
    for (int part = 0; part < 2; part++) {
        const int tau = (fe ? 0 : 2) + part;
        const real *cA = C + P_CA + tau * NA * NB, *cS = C + P_CSA + tau * NA * NB;
        const bool spins = FE && part == 0;
        const int b = part ? nfe : 0, e = part ? cnt : nfe;
        // this lane's neighbour index two rounds ahead, its position one round ahead
        int jc = b + lane < e ? S.nbrA[(size_t)(b + lane) * ld + i] : 0;
        int jn = b + lane + 8 < e ? S.nbrA[(size_t)(b + lane + 8) * ld + i] : jc;
        d4 pc = S.pos[jc];
#pragma unroll 1
        for (int base = b; base < e; base += 8) {
            const int s0 = base + lane;
            int j0 = jc;
            const d4 pj = pc;
            jc = jn;
            pc = S.pos[jc];
            if (s0 + 16 < e) jn = S.nbrA[(size_t)(s0 + 16) * ld + i];
            real d0[3] = {0, 0, 0}, r20 = rc2;
            if (s0 < e) r20 = geom_p(R, pi, pj, d0);
            else j0 = 0;
            const bool in = s0 < e && r20 < rc2;
            // records of listed pairs beyond the cutoff are zero; each record
            // goes where the partner's gather reads it
            if (s0 < e && !in) {
                real *z = W.pbA + ((size_t)S.revA[s0 * ld + i] * ld + j0) * 4;
                z[0] = z[1] = z[2] = z[3] = 0;
            }
            const unsigned gm = (unsigned)(__ballot(in) >> gbase) & 0xffu;
            const int c = __popc(gm);
            const int q = (lane - rank) & 7;
            int src = 0;
            {
                unsigned m = gm;
                for (int x = 0; x < q && m; x++) m &= m - 1;
                src = m ? __ffs(m) - 1 : 0;
            }
            const bool mine = q < c;
            rank += c;
            const int j = __shfl(j0, gbase + src);
            const int s = __shfl(s0, gbase + src);
            real d[3];
            d[0] = __shfl(d0[0], gbase + src);
            d[1] = __shfl(d0[1], gbase + src);
            d[2] = __shfl(d0[2], gbase + src);
            const real r2 = __shfl(r20, gbase + src);
            if (!mine) continue;
            real *rec = W.pbA + ((size_t)S.revA[s * ld + i] * ld + j) * 4;
            real r, ir;
            r_and_inv(r2, r, ir);
            const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
            real f[NB], df[NB];
            radial_basis_d(r, rc, f, df);
            real sig = 0, sj[3] = {0, 0, 0};
            if (spins) {
                load_spin(S.spin, j, sj);
                sig = si[0] * sj[0] + si[1] * sj[1] + si[2] * sj[2];
            }
            real gA[NA], dgA[NA], gS[NA], dgS[NA];
#pragma unroll
            for (int n = 0; n < NA; n++) {
                gA[n] = dotc(cA + n * NB, f);
                dgA[n] = dotc(cA + n * NB, df);
                gS[n] = spins ? dotc(cS + n * NB, f) : real(0);
                dgS[n] = spins ? dotc(cS + n * NB, df) : real(0);
            }
            real sv = 0, sl = 0, hs = 0, su0 = 0, su1 = 0, su2 = 0;
            // straight-line over the 24 harmonics; the register fence before
            // each one keeps the compiler from evaluating all of them at once
            static_for<NLM>([&](auto M) {
                constexpr int m = decltype(M)::value;
                real Y, gx, gy, gz;
                real hx = rh[0], hy = rh[1], hz = rh[2];
                int qo = slot * QSTRIDE;
                asm volatile("" : "+v"(hx), "+v"(hy), "+v"(hz), "+v"(qo), "+v"(sv), "+v"(sl), "+v"(hs), "+v"(su0),
                             "+v"(su1), "+v"(su2));
                const real *Qm = sQ + qo;
                harmonic_one<m>(hx, hy, hz, Y, gx, gy, gz);
                real qa_g = 0, qa_dg = 0, qs_g = 0, qs_dg = 0;
#pragma unroll
                for (int n = 0; n < NA; n++) {
                    const real qa = Qm[n * NLM + m];
                    qa_g += qa * gA[n];
                    qa_dg += qa * dgA[n];
                }
                if (FE && spins) {
#pragma unroll
                    for (int n = 0; n < NA; n++) {
                        const real qs = Qm[NA * NLM + n * NLM + m];
                        qs_g += qs * gS[n];
                        qs_dg += qs * dgS[n];
                    }
                }
                const real U = qa_g + sig * qs_g, V = qa_dg + sig * qs_dg;
                sv += V * Y;
                sl += real(l_of_lm(m)) * U * Y;
                hs += qs_g * Y;
                su0 += U * gx;
                su1 += U * gy;
                su2 += U * gz;
            });
            const real G0 = sv * rh[0] + (su0 - sl * rh[0]) * ir;
            const real G1 = sv * rh[1] + (su1 - sl * rh[1]) * ir;
            const real G2 = sv * rh[2] + (su2 - sl * rh[2]) * ir;
            rec[0] = G0;
            rec[1] = G1;
            rec[2] = G2;
            rec[3] = hs;
            Fo[0] += G0;
            Fo[1] += G1;
            Fo[2] += G2;
            ho[0] += hs * sj[0];
            ho[1] += hs * sj[1];
            ho[2] += hs * sj[2];
        }
    }
    // own-side sums over the atom's eight lanes (fixed xor tree)
#pragma unroll
    for (int x = 0; x < 3; x++) {
        Fo[x] = xor_sum8(Fo[x]);
        ho[x] = xor_sum8(ho[x]);
    }
    if (lane == 0) put_pair(W.ownA, (size_t)i, Fo, ho);
}

// -------------------------------------------------------------------------
// gather: forces and fields
// -------------------------------------------------------------------------

template <typename real>
__global__ void __launch_bounds__(256) k_gather(Sys S, Work<real> W) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= S.N || live(S, k) < 0) return;   // a paused replica keeps its last forces and fields
    const size_t ld = S.N;
    const bool fe = S.mag && k < S.N_fe;   // spin carrier
    real F[3], h[3];
    {
        const real *a = W.ownR + (size_t)k * 6;
        F[0] = a[0];
        F[1] = a[1];
        F[2] = a[2];
        h[0] = a[3];
        h[1] = a[4];
        h[2] = a[5];
    }
    const int na = S.cntA[k];
    {
        const real *a = W.ownA + (size_t)k * 6;
        F[0] += a[0];
        F[1] += a[1];
        F[2] += a[2];
        h[0] += a[3];
        h[1] += a[4];
        h[2] += a[5];
    }
    // partner records sit in this atom's own slots: the reads are coalesced
    if (fe) {
        const real *a = W.ownM + (size_t)k * 6;
        F[0] += a[0];
        F[1] += a[1];
        F[2] += a[2];
        h[0] += a[3];
        h[1] += a[4];
        h[2] += a[5];
    }
#pragma unroll 4
    for (int s = 0; s < na; s++) {
        const real *p = W.pbA + ((size_t)s * ld + k) * 4;
        F[0] -= p[0];
        F[1] -= p[1];
        F[2] -= p[2];
        if (fe) {
            const int j = S.nbrA[s * ld + k];
            if (j < S.N_fe) {
                real sj[3];
                load_spin(S.spin, j, sj);
                h[0] += p[3] * sj[0];
                h[1] += p[3] * sj[1];
                h[2] += p[3] * sj[2];
            }
        }
    }
    d4 f4 = {(double)F[0], (double)F[1], (double)F[2], 0.0};
    S.force[k] = f4;
    d4 h4 = {0, 0, 0, 0};
    if (fe) {
        const RepDev &R = S.rep[S.rid[k]];
        const double fr = ramp_frac(R), zs = R.mu_s * MUB;
        h4.x = -(double)h[0] + zs * (R.B0[0] + (R.B1[0] - R.B0[0]) * fr);
        h4.y = -(double)h[1] + zs * (R.B0[1] + (R.B1[1] - R.B0[1]) * fr);
        h4.z = -(double)h[2] + zs * (R.B0[2] + (R.B1[2] - R.B0[2]) * fr);
    }
    S.field[k] = h4;
}

// -------------------------------------------------------------------------
// spin couplings of the frozen-Fp magnetic energy
//   E_lin = sum_i sum_j [a_ij s_i.s_j + d_ij rhat_ij.(s_i x s_j) + b_ij (s_i.rhat)(s_j.rhat)]
//           + sum_i s_i^T A_i s_i + o_i |s_i|^2  (+ Zeeman)
// -------------------------------------------------------------------------

// spin-angular part of a_ij: sum_n g^sa_n(r_ij) sum_lm Fp^sa_nl A_nlm Y_lm(rhat_ij);
// lanes take the atom's spin-carrying neighbours round robin, P = Fp^sa A in LDS
constexpr int PSTRIDE = NA * NLM + 1;

template <typename real>
__global__ void __launch_bounds__(64) k_assemble_angular(Sys S, const real *__restrict__ C, Work<real> W) {
    __shared__ real sP[ANG_ATOMS * PSTRIDE];
    const int lane = threadIdx.x & 7, slot = threadIdx.x >> 3;
    const int i0 = blockIdx.x * ANG_ATOMS + slot;
    const int i = live(S, i0 < S.N_fe ? i0 : -1);
    const real *cS = C + P_CSA;   // tau = (Fe, Fe)
    real *P = sP + slot * PSTRIDE;
    if (i >= 0) {
        const real *Fp = W.Fp + (size_t)i * DP;
        for (int x = lane; x < NA * NLM; x += 8) {
            const int n = x / NLM, m = x - n * NLM;
            P[x] = Fp[D_SA + 4 * n + l_of_lm(m) - 1] * W.AB[((size_t)i * NA + n) * NAB + m];
        }
    }
    __syncthreads();
    if (i < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_A, rc2 = rc * rc;
    const int nfe = S.cntFeA[i];
    const size_t ld = S.N, lf = S.N_fe;
    // this lane's neighbour index two rounds ahead, its position one round ahead
    int j1 = lane < nfe ? S.nbrA[(size_t)lane * ld + i] : 0;
    int j2 = lane + 8 < nfe ? S.nbrA[(size_t)(lane + 8) * ld + i] : j1;
    d4 p1 = S.pos[j1];
    for (int s = lane; s < nfe; s += 8) {
        const d4 pj = p1;
        j1 = j2;
        p1 = S.pos[j1];
        if (s + 16 < nfe) j2 = S.nbrA[(size_t)(s + 16) * ld + i];
        real d[3];
        const real r2 = geom_p(R, pi, pj, d);
        if (r2 >= rc2) continue;
        real r, ir;
        r_and_inv(r2, r, ir);
        real f[NB];
        radial_basis(r, rc, f);
        real gS[NA];
#pragma unroll
        for (int n = 0; n < NA; n++) gS[n] = dotc(cS + n * NB, f);
        real a = 0;
        real Y[NLM];
        harmonics(d[0] * ir, d[1] * ir, d[2] * ir, Y);
#pragma unroll
        for (int m = 0; m < NLM; m++) {
            real w = 0;
#pragma unroll
            for (int n = 0; n < NA; n++) w += P[n * NLM + m] * gS[n];
            a += w * Y[m];
        }
        const int sr = S.a2r[s * ld + i];
        if (sr < MAXFE) W.csa[(size_t)sr * lf + i] = a;
    }
}

// Couplings of the spin-carrying pairs inside rc_R, J_ij = a_ij + a_ji,
// D_ij = d_ij + d_ji, K_ij = b_ij + b_ji: the radial-set parts are sums over
// the basis with the summed contracted coefficients of both spins, the
// spin-angular parts (inside rc_A) the two atoms' records. Stored with rhat_ij
// compactly in list order, so the sweep's split of a spin's couplings over
// lanes depends on the positions alone and not on which farther atoms the
// Verlet list happens to hold. The same pass sums the single-ion tensor
// A_i = sum_j g^si(r_ij) rhat rhat^T over all neighbours.
template <typename real>
__global__ void __launch_bounds__(256) k_assemble_pairs(Sys S, const real *__restrict__ C, Work<real> W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe || live(S, i) < 0) return;
    const Img R = img_of(S.rep[S.rid[i]]);
    const d4 pi = S.pos[i];
    const real rc = (real)RC_R, rc2 = rc * rc, rca = (real)RC_A, rca2 = rca * rca;   // as the angular pass
    const int cnt = S.cntR[i], nfe_all = S.cntFeR[i], nfe = min(nfe_all, MAXFE);
    const size_t ld = S.N, lf = S.N_fe;
    const int p = S.colpos[i];
    const real *Fp = W.Fp + (size_t)i * DP;
    real Ci[MCOEF];
    {
        const real *m = W.mcoef + (size_t)i * MCOEF;
#pragma unroll
        for (int k = 0; k < MCOEF; k++) Ci[k] = m[k];
    }
    real Axx = 0, Ayy = 0, Azz = 0, Axy = 0, Axz = 0, Ayz = 0;
    int cs = 0;
    {
        real CS[NB];
        contract((C + P_CSI), Fp + D_SI, NR, CS);
        // neighbour index two slots ahead, its position one slot ahead
        int j1 = 0 < nfe ? S.nbrR[i] : 0;
        int j2 = 1 < nfe ? S.nbrR[ld + i] : j1;
        d4 p1 = S.pos[j1];
        // first the in-cutoff slots (nfe <= MAXFE = 64 bits), then the work in
        // slot order over those alone: at temperature the lanes of a
        // wavefront have their out-of-cutoff slots at different places, and
        // a loop over all slots would run its body for their union
        uint64_t in = 0;
        for (int s = 0; s < nfe; s++) {
            const d4 pj = p1;
            j1 = j2;
            p1 = S.pos[j1];
            if (s + 2 < nfe) j2 = S.nbrR[(size_t)(s + 2) * ld + i];
            real d[3];
            if (geom_p(R, pi, pj, d) < rc2) in |= 1ull << s;
        }
        int s = in ? __ffsll((long long)in) - 1 : -1;
        in = in ? in & (in - 1) : 0;
        int jn = s >= 0 ? S.nbrR[(size_t)s * ld + i] : 0;
        d4 pn = S.pos[jn];
        while (s >= 0) {
            const int j = jn;
            const d4 pj = pn;
            const int s_ = s;
            s = in ? __ffsll((long long)in) - 1 : -1;
            in = in ? in & (in - 1) : 0;
            if (s >= 0) {
                jn = S.nbrR[(size_t)s * ld + i];
                pn = S.pos[jn];
            }
            real d[3];
            const real r2 = geom_p(R, pi, pj, d);
            real r, ir;
            r_and_inv(r2, r, ir);
            const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
            real f[NB];
            radial_basis(r, rc, f);
            const real *mj = W.mcoef + (size_t)j * MCOEF;
            real J = 0, D = 0, K = 0;
#pragma unroll
            for (int k = 0; k < NB; k++) {
                J += (Ci[k] + mj[k]) * f[k];
                D += (Ci[NB + k] + mj[NB + k]) * f[k];
                K += (Ci[2 * NB + k] + mj[2 * NB + k]) * f[k];
            }
            if (r2 < rca2) {
                const int t = min(S.revR[s_ * ld + i], MAXFE - 1);
                J += W.csa[(size_t)s_ * lf + i] + W.csa[(size_t)t * lf + j];
            }
            const real g = dotk(CS, f);
            Axx += g * rh[0] * rh[0];
            Ayy += g * rh[1] * rh[1];
            Azz += g * rh[2] * rh[2];
            Axy += g * rh[0] * rh[1];
            Axz += g * rh[0] * rh[2];
            Ayz += g * rh[1] * rh[2];
            real *c = W.cpl + ((size_t)cs * lf + p) * 6;
            c[0] = J;
            c[1] = D;
            c[2] = K;
            c[3] = rh[0];
            c[4] = rh[1];
            c[5] = rh[2];
            W.cpl_j[(size_t)cs * lf + p] = j;
            cs++;
        }
    }
    {
        real CS[NB];
        contract((C + P_CSI) + 1 * NR * NB, Fp + D_SI, NR, CS);
        int j1 = nfe_all < cnt ? S.nbrR[(size_t)nfe_all * ld + i] : 0;
        int j2 = nfe_all + 1 < cnt ? S.nbrR[(size_t)(nfe_all + 1) * ld + i] : j1;
        d4 p1 = S.pos[j1];
        for (int s = nfe_all; s < cnt; s++) {
            const d4 pj = p1;
            j1 = j2;
            p1 = S.pos[j1];
            if (s + 2 < cnt) j2 = S.nbrR[(size_t)(s + 2) * ld + i];
            real d[3];
            const real r2 = geom_p(R, pi, pj, d);
            if (r2 >= rc2) continue;
            real r, ir;
            r_and_inv(r2, r, ir);
            const real rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
            real f[NB];
            radial_basis(r, rc, f);
            const real g = dotk(CS, f);
            Axx += g * rh[0] * rh[0];
            Ayy += g * rh[1] * rh[1];
            Azz += g * rh[2] * rh[2];
            Axy += g * rh[0] * rh[1];
            Axz += g * rh[0] * rh[2];
            Ayz += g * rh[1] * rh[2];
        }
    }
    real *o = W.selfc + (size_t)p * 8;
    o[0] = Axx;
    o[1] = Ayy;
    o[2] = Azz;
    o[3] = Axy;
    o[4] = Axz;
    o[5] = Ayz;
    o[6] = Fp[D_OS];
    o[7] = 0;
    W.cpl_n[p] = cs;
}

inline int nblk(int n, int b) { return (n + b - 1) / b; }

}  // namespace

#define NEP_SPLIT(per)                                  \
    const int ge = S.N - S.N_fe;                        \
    const int nb_fe = nblk(S.N_fe, per), nb_ge = nblk(ge, per);

// spin-step passes (PASS_SPIN, PASS_SPIN_REUSE) cover the spin carriers only:
// the frozen-Fp magnetic energy has no term on atoms without a spin
template <typename real>
void launch_desc_radial(const Sys &S, const ModelDev<real> &M, const Work<real> &W, const d4 *spin, int mode,
                        hipStream_t st) {
    if (S.N == 0) return;
    NEP_SPLIT(256)
    const int nb = mode == PASS_FULL ? nb_fe + nb_ge : nb_fe;
    if (nb) hipLaunchKernelGGL(k_desc_radial<real>, dim3(nb), dim3(256), 0, st, S, M.cR, W, spin, nb_fe);
}

template <typename real>
void launch_desc_angular(const Sys &S, const ModelDev<real> &M, const Work<real> &W, const d4 *spin, int mode,
                         hipStream_t st) {
    if (S.N == 0) return;
    NEP_SPLIT(ANG_ATOMS)
    const int nb = mode == PASS_FULL ? nb_fe + nb_ge : nb_fe;
    if (nb)
        hipLaunchKernelGGL(k_desc_angular<real>, dim3(nb), dim3(8 * ANG_ATOMS), 0, st, S, M.cR, W, spin, nb_fe, mode);
}

template <typename real>
void launch_mlp(const Sys &S, const ModelDev<real> &M, const Work<real> &W, int mode, hipStream_t st) {
    if (S.N == 0) return;
    NEP_SPLIT(MLP_ATOMS)
    const int nb = mode == PASS_FULL ? nb_fe + nb_ge : nb_fe;
    if (!nb) return;
    if (S.mag) hipLaunchKernelGGL((k_mlp<real, DP>), dim3(nb), dim3(64 * MLP_WAVES), 0, st, S, M, W, nb_fe);
    else hipLaunchKernelGGL((k_mlp<real, DS_PAD>), dim3(nb), dim3(64 * MLP_WAVES), 0, st, S, M, W, nb_fe);
}

template <typename real>
void launch_bwd_radial(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st) {
    if (S.N == 0) return;
    NEP_SPLIT(256)
    hipLaunchKernelGGL(k_radial_coef<real>, dim3(nblk(S.N, 256)), dim3(256), 0, st, S, M.cR, W);
    hipLaunchKernelGGL(k_bwd_radial<real>, dim3(nb_fe + nb_ge), dim3(256), 0, st, S, M.cR, W, nb_fe);
    if (nb_fe && S.mag) hipLaunchKernelGGL(k_bwd_mag<real>, dim3(nb_fe), dim3(256), 0, st, S, M.cR, W);
}

template <typename real>
void launch_bwd_angular(const Sys &S, const ModelDev<real> &M, const Work<real> &W, int species, hipStream_t st) {
    if (S.N == 0) return;
    NEP_SPLIT(ANG_ATOMS)
    if (species == 0 && nb_fe) {
        if (S.mag)
            hipLaunchKernelGGL((k_bwd_angular<real, true>), dim3(nb_fe), dim3(8 * ANG_ATOMS), 0, st, S, M.cR, W, 0,
                               S.N_fe);
        else
            hipLaunchKernelGGL((k_bwd_angular<real, false>), dim3(nb_fe), dim3(8 * ANG_ATOMS), 0, st, S, M.cR, W, 0,
                               S.N_fe);
    }
    if (species == 1 && nb_ge)
        hipLaunchKernelGGL((k_bwd_angular<real, false>), dim3(nb_ge), dim3(8 * ANG_ATOMS), 0, st, S, M.cR, W, S.N_fe,
                           S.N);
}

template <typename real>
void launch_gather(const Sys &S, const Work<real> &W, hipStream_t st) {
    if (S.N == 0) return;
    hipLaunchKernelGGL(k_gather<real>, dim3(nblk(S.N, 256)), dim3(256), 0, st, S, W);
}

template <typename real>
void launch_assemble_coef(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st) {
    if (S.N_fe == 0) return;
    hipLaunchKernelGGL(k_mag_coef<real>, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S, M.cR, W);
    hipLaunchKernelGGL(k_assemble_angular<real>, dim3(nblk(S.N_fe, ANG_ATOMS)), dim3(8 * ANG_ATOMS), 0, st, S, M.cR, W);
}

template <typename real>
void launch_assemble_pairs(const Sys &S, const ModelDev<real> &M, const Work<real> &W, hipStream_t st) {
    if (S.N_fe == 0) return;
    hipLaunchKernelGGL(k_assemble_pairs<real>, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S, M.cR, W);
}

#define NEP_INST(real)                                                                                           \
    template void launch_desc_radial<real>(const Sys &, const ModelDev<real> &, const Work<real> &, const d4 *, \
                                           int, hipStream_t);                                                    \
    template void launch_desc_angular<real>(const Sys &, const ModelDev<real> &, const Work<real> &, const d4 *,\
                                            int, hipStream_t);                                                   \
    template void launch_mlp<real>(const Sys &, const ModelDev<real> &, const Work<real> &, int, hipStream_t);   \
    template void launch_bwd_radial<real>(const Sys &, const ModelDev<real> &, const Work<real> &, hipStream_t); \
    template void launch_bwd_angular<real>(const Sys &, const ModelDev<real> &, const Work<real> &, int, hipStream_t);\
    template void launch_gather<real>(const Sys &, const Work<real> &, hipStream_t);                             \
    template void launch_assemble_coef<real>(const Sys &, const ModelDev<real> &, const Work<real> &, hipStream_t);\
    template void launch_assemble_pairs<real>(const Sys &, const ModelDev<real> &, const Work<real> &, hipStream_t);

NEP_INST(double)
NEP_INST(float)

}  // namespace nep
