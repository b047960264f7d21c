// common.h -- types, constants and device helpers shared by the HIP kernels
// of the spin-lattice NEP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace nep {

// model sizes (descriptor layout of the spin-aware NEP, Sec. 5.1)
constexpr int NR = 9;      // radial-set functions n = 0..8
constexpr int NA = 7;      // angular-set functions n = 0..6
constexpr int NB = 9;      // Chebyshev basis T_0..T_8 (basis size 8, Sec. 5.2)
constexpr int NH = 64;     // hidden units per species
constexpr int ND = 102;    // descriptor length
constexpr int DP = 104;    // padded descriptor row
// the structural-only NEP (no magnetic channels): q^R and q^A, the first 37
// entries of the same row; its read-out contracts over 40 (a multiple of 4)
constexpr int DS = 37, DS_PAD = 40;
constexpr int N_PARAMS_STRUCT = 324 + 252 + 2 * (NH * DS + NH + NH + 1);
constexpr int NLM = 24;    // real harmonics l = 1..4
constexpr int NAB = 2 * NLM;   // angular accumulators per (atom, n): A then B

constexpr int D_R = 0, D_A = 9, D_OS = 37, D_EX = 38, D_DM = 47, D_AN = 56, D_SI = 65, D_SA = 74;

constexpr int P_CR = 0, P_CA = 324, P_CEX = 576, P_CDM = 900, P_CAN = 1224, P_CSI = 1548,
              P_CSA = 1872, P_MLP = 2124, P_MLP_STRIDE = 6657, N_PARAMS = 15438;

constexpr int MAXR = 160;  // listed neighbours within rc_R + skin (liquid water at skin 0.5: ~115)
constexpr int MAXA = 96;   // listed neighbours within rc_A + skin

constexpr double RC_R = 6.0;
constexpr double RC_A = 4.5;

// metal units: A, eV, fs, u, K, T
constexpr double KAPPA = 9.648533212e-3;
constexpr double KB = 8.617333262e-5;
constexpr double HBAR = 0.6582119569;
constexpr double MUB = 5.7883818060e-5;
constexpr double PI = 3.14159265358979323846;

// default masses of the two species (Fe, Ge)
__host__ __device__ inline double mass_of(int t) { return t == 0 ? 55.845 : 72.630; }

struct alignas(32) d4 {
    double x, y, z, w;
};

// Per-replica parameters, resident in device memory. Every kernel finds its
// atom's replica through rid[] and reads box, schedule and counters here.
struct RepDev {
    double box[3], ibox[3];
    double dt, T0, T1, alpha, gammaL, mu_s, mid_tol, skin;
    double B0[3], B1[3];
    double cell_lo[3], cell_w[3];
    long long n_ramp, step, step_end;
    unsigned long long seed;
    int pbc[3], nc[3];
    int ensemble, mid_cap, active, failed;
    int cell_base, n_atoms, fe_off, n_fe, ge_off, n_ge;
    double mass[2];                 // per species (u)
    double sc_tol;                  // self-consistent midpoint tolerance (0: fixed K_corr)
    unsigned long long sc_delta;    // max |S^(p) - S^(p-1)| of the current pass, as bits
    int sc_max, sc_done;            // pass cap; converged in this step
    double landau_a, landau_b;      // the model's onsite moment-length term a|s|^2 + b|s|^4
    double lsf_gamma;               // damping of the longitudinal spin dynamics
    int lsf;                        // 1: spins of variable length (longitudinal Langevin dynamics)
    int capped;                     // rotations of this step stopped at mid_cap without meeting mid_tol
    int sc_passes;                  // sweep passes of the last spin step (self-consistent batches)
    double sc_last;                 // and the change of its last pass
};

__device__ inline double ramp_frac(const RepDev &R) {
    if (R.n_ramp <= 0) return 0.0;
    long long n = R.step < R.n_ramp ? R.step : R.n_ramp;
    return (double)n / (double)R.n_ramp;
}

// minimum-image displacement d = pj - pi (FP64 always)
__device__ inline void min_image(const RepDev &R, const d4 &pi, const d4 &pj, double &dx, double &dy,
                                 double &dz) {
    dx = pj.x - pi.x;
    dy = pj.y - pi.y;
    dz = pj.z - pi.z;
    if (R.pbc[0]) dx -= R.box[0] * rint(dx * R.ibox[0]);
    if (R.pbc[1]) dy -= R.box[1] * rint(dy * R.ibox[1]);
    if (R.pbc[2]) dz -= R.box[2] * rint(dz * R.ibox[2]);
}

// The box of one replica in registers for neighbour loops: free axes carry a
// zero edge and inverse edge, so the correction box * rint(d * ibox) is an
// exact zero there and the loop needs neither branches nor reloads of the
// replica record.
struct Img {
    double b[3], ib[3];
};
__device__ inline Img img_of(const RepDev &R) {
    Img g;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        g.b[a] = R.pbc[a] ? R.box[a] : 0.0;
        g.ib[a] = R.pbc[a] ? R.ibox[a] : 0.0;
    }
    return g;
}
__device__ inline void min_image(const Img &g, const d4 &pi, const d4 &pj, double &dx, double &dy, double &dz) {
    dx = pj.x - pi.x;
    dy = pj.y - pi.y;
    dz = pj.z - pi.z;
    dx -= g.b[0] * rint(dx * g.ib[0]);
    dy -= g.b[1] * rint(dy * g.ib[1]);
    dz -= g.b[2] * rint(dz * g.ib[2]);
}

template <typename real>
__device__ inline real dcos(real x);
template <>
__device__ inline double dcos<double>(double x) { return cos(x); }
template <>
__device__ inline float dcos<float>(float x) { return cosf(x); }
template <typename real>
__device__ inline real dsin(real x);
template <>
__device__ inline double dsin<double>(double x) { return sin(x); }
template <>
__device__ inline float dsin<float>(float x) { return sinf(x); }
template <typename real>
__device__ inline real dsqrt(real x);
template <>
__device__ inline double dsqrt<double>(double x) { return sqrt(x); }
template <>
__device__ inline float dsqrt<float>(float x) { return sqrtf(x); }
template <typename real>
__device__ inline real dexp(real x);
template <>
__device__ inline double dexp<double>(double x) { return exp(x); }
template <>
__device__ inline float dexp<float>(float x) { return expf(x); }

template <typename real>
__device__ inline real dtanh(real x);
template <>
__device__ inline double dtanh<double>(double x) { return tanh(x); }
template <>
__device__ inline float dtanh<float>(float x) { return tanhf(x); }

// Cutoff function fc(r) = (1 + cos(pi r/rc))/2 and its r-derivative. With
// t = pi (r/rc - 1/2), |t| <= pi/2: cos(pi r/rc) = -sin t and
// sin(pi r/rc) = cos t. In FP64 sin t and cos t come from their Taylor series
// (coefficients +-1/n!, truncation below 2e-18 on |t| <= pi/2); FP32 uses
// the device sinf/cosf.
__device__ inline void sin_cos_halfpi(double t, double &sn, double &cs) {
    const double t2 = t * t;
    // p = -(1 - t^2/3! + t^4/5! - ... + t^20/21!), so sin t = -t p
    double p = -1.0 / 51090942171709440000.0;           // 21!
    p = p * t2 + 1.0 / 121645100408832000.0;            // 19!
    p = p * t2 - 1.0 / 355687428096000.0;               // 17!
    p = p * t2 + 1.0 / 1307674368000.0;                 // 15!
    p = p * t2 - 1.0 / 6227020800.0;                    // 13!
    p = p * t2 + 1.0 / 39916800.0;                      // 11!
    p = p * t2 - 1.0 / 362880.0;                        // 9!
    p = p * t2 + 1.0 / 5040.0;                          // 7!
    p = p * t2 - 1.0 / 120.0;                           // 5!
    p = p * t2 + 1.0 / 6.0;                             // 3!
    p = p * t2 - 1.0;
    sn = -t * p;
    // q = 1/2! - t^2/4! + ... + t^20/22!, so cos t = 1 - t^2 q
    double q = 1.0 / 1124000727777607680000.0;          // 1/22!
    q = q * t2 - 1.0 / 2432902008176640000.0;           // -1/20!
    q = q * t2 + 1.0 / 6402373705728000.0;              // 1/18!
    q = q * t2 - 1.0 / 20922789888000.0;                // -1/16!
    q = q * t2 + 1.0 / 87178291200.0;                   // 1/14!
    q = q * t2 - 1.0 / 479001600.0;                     // -1/12!
    q = q * t2 + 1.0 / 3628800.0;                       // 1/10!
    q = q * t2 - 1.0 / 40320.0;                         // -1/8!
    q = q * t2 + 1.0 / 720.0;                           // 1/6!
    q = q * t2 - 1.0 / 24.0;                            // -1/4!
    q = q * t2 + 0.5;                                   // 1/2!
    cs = 1.0 - t2 * q;
}

template <typename real>
__device__ inline void cutoff_fc(real r, real rc, real &fc, real &dfc);
template <>
__device__ inline void cutoff_fc<double>(double r, double rc, double &fc, double &dfc) {
    const double irc = 1.0 / rc;    // rc is a constant at every call site: folded
    double sn, cs;
    sin_cos_halfpi(PI * (r * irc - 0.5), sn, cs);
    fc = 0.5 * (1.0 - sn);
    dfc = (-0.5 * PI * irc) * cs;
}
template <>
__device__ inline void cutoff_fc<float>(float r, float rc, float &fc, float &dfc) {
    const float a = (float)PI / rc;
    fc = 0.5f * (1.0f + cosf(a * r));
    dfc = -0.5f * a * sinf(a * r);
}

// r and 1/r from r^2: hardware reciprocal square root refined by Newton steps
template <typename real>
__device__ inline void r_and_inv(real r2, real &r, real &ir);
template <>
__device__ inline void r_and_inv<double>(double r2, double &r, double &ir) {
    double y = __builtin_amdgcn_rsq(r2);
    y = y * (1.5 - 0.5 * r2 * y * y);
    y = y * (1.5 - 0.5 * r2 * y * y);
    ir = y;
    r = r2 * y;
}
template <>
__device__ inline void r_and_inv<float>(float r2, float &r, float &ir) {
    ir = rsqrtf(r2);
    r = r2 * ir;
}

// Chebyshev radial basis at r < rc: f_k = (T_k(x)+1)/2 * fc(r), x = 2(r/rc-1)^2-1,
// with T_k by the running recurrence T_{k+1} = 2x T_k - T_{k-1}.
template <typename real>
__device__ inline void radial_basis(real r, real rc, real f[NB]) {
    real fc, dfc;
    cutoff_fc(r, rc, fc, dfc);
    const real u = r * (real(1) / rc) - real(1);
    const real x = real(2) * u * u - real(1);
    real t0 = real(1), t1 = x;
    const real hf = real(0.5) * fc;
    f[0] = fc;
    f[1] = (t1 + real(1)) * hf;
#pragma unroll
    for (int k = 2; k < NB; k++) {
        real t2 = real(2) * x * t1 - t0;
        f[k] = (t2 + real(1)) * hf;
        t0 = t1;
        t1 = t2;
    }
}

// basis and its r-derivative; dT_{k+1} = 2 T_k + 2x dT_k - dT_{k-1}
template <typename real>
__device__ inline void radial_basis_d(real r, real rc, real f[NB], real df[NB]) {
    real fc, dfc;
    cutoff_fc(r, rc, fc, dfc);
    const real u = r * (real(1) / rc) - real(1);
    const real x = real(2) * u * u - real(1);
    const real dx = real(4) * u * (real(1) / rc);
    real t0 = real(1), t1 = x, d0 = real(0), d1 = real(1);
    f[0] = fc;
    df[0] = dfc;
    f[1] = real(0.5) * (t1 + real(1)) * fc;
    df[1] = real(0.5) * (d1 * dx * fc + (t1 + real(1)) * dfc);
#pragma unroll
    for (int k = 2; k < NB; k++) {
        real t2 = real(2) * x * t1 - t0;
        real d2 = real(2) * t1 + real(2) * x * d1 - d0;
        f[k] = real(0.5) * (t2 + real(1)) * fc;
        df[k] = real(0.5) * (d2 * dx * fc + (t2 + real(1)) * dfc);
        t0 = t1;
        t1 = t2;
        d0 = d1;
        d1 = d2;
    }
}

// Real solid harmonics R_lm of degree l = 1..4 normalised so that
// sum_m R_lm(a) R_lm(b) = P_l(a.b) for unit a, b (addition theorem);
// evaluated at a unit vector (x, y, z). Order: l = 1 (3), l = 2 (5),
// l = 3 (7), l = 4 (9).
template <typename real>
__device__ inline void harmonics(real x, real y, real z, real Y[NLM]) {
    const real s3 = real(1.7320508075688772), s38 = real(0.61237243569579452),
               s15h = real(1.9364916731037085), s15 = real(3.8729833462074170),
               s58 = real(0.79056941504209483), s10q = real(0.79056941504209483),
               s5q = real(0.55901699437494742), s5h = real(1.1180339887498949),
               s70q = real(2.0916500663351889), s35e = real(0.73950997288745200),
               s35h = real(2.9580398915498080);
    const real xx = x * x, yy = y * y, zz = z * z, p2 = xx + yy;
    Y[0] = x;
    Y[1] = y;
    Y[2] = z;
    Y[3] = s3 * x * y;
    Y[4] = s3 * y * z;
    Y[5] = real(0.5) * (real(2) * zz - p2);
    Y[6] = s3 * x * z;
    Y[7] = real(0.5) * s3 * (xx - yy);
    Y[8] = z * (zz - real(1.5) * p2);
    Y[9] = s38 * x * (real(4) * zz - p2);
    Y[10] = s38 * y * (real(4) * zz - p2);
    Y[11] = s15h * z * (xx - yy);
    Y[12] = s15 * x * y * z;
    Y[13] = s58 * x * (xx - real(3) * yy);
    Y[14] = s58 * y * (real(3) * xx - yy);
    Y[15] = zz * zz - real(3) * zz * p2 + real(0.375) * p2 * p2;
    Y[16] = s10q * x * z * (real(4) * zz - real(3) * p2);
    Y[17] = s10q * y * z * (real(4) * zz - real(3) * p2);
    Y[18] = s5q * (xx - yy) * (real(6) * zz - p2);
    Y[19] = s5h * x * y * (real(6) * zz - p2);
    Y[20] = s70q * x * z * (xx - real(3) * yy);
    Y[21] = s70q * y * z * (real(3) * xx - yy);
    Y[22] = s35e * (xx * xx - real(6) * xx * yy + yy * yy);
    Y[23] = s35h * x * y * (xx - yy);
}

// gradients of the homogeneous polynomials R_lm at (x, y, z)
template <typename real>
__device__ inline void harmonics_grad(real x, real y, real z, real G[NLM][3]) {
    const real s3 = real(1.7320508075688772), s38 = real(0.61237243569579452),
               s15h = real(1.9364916731037085), s15 = real(3.8729833462074170),
               s58 = real(0.79056941504209483), s10q = real(0.79056941504209483),
               s5 = real(2.2360679774997897), s5h = real(1.1180339887498949),
               s70q = real(2.0916500663351889), s35e = real(0.73950997288745200),
               s35h = real(2.9580398915498080);
    const real xx = x * x, yy = y * y, zz = z * z, p2 = xx + yy;
    G[0][0] = 1; G[0][1] = 0; G[0][2] = 0;
    G[1][0] = 0; G[1][1] = 1; G[1][2] = 0;
    G[2][0] = 0; G[2][1] = 0; G[2][2] = 1;
    G[3][0] = s3 * y; G[3][1] = s3 * x; G[3][2] = 0;
    G[4][0] = 0; G[4][1] = s3 * z; G[4][2] = s3 * y;
    G[5][0] = -x; G[5][1] = -y; G[5][2] = real(2) * z;
    G[6][0] = s3 * z; G[6][1] = 0; G[6][2] = s3 * x;
    G[7][0] = s3 * x; G[7][1] = -s3 * y; G[7][2] = 0;
    G[8][0] = real(-3) * x * z; G[8][1] = real(-3) * y * z; G[8][2] = real(3) * zz - real(1.5) * p2;
    G[9][0] = s38 * (real(4) * zz - real(3) * xx - yy); G[9][1] = s38 * real(-2) * x * y; G[9][2] = s38 * real(8) * x * z;
    G[10][0] = s38 * real(-2) * x * y; G[10][1] = s38 * (real(4) * zz - xx - real(3) * yy); G[10][2] = s38 * real(8) * y * z;
    G[11][0] = s15 * x * z; G[11][1] = -s15 * y * z; G[11][2] = s15h * (xx - yy);
    G[12][0] = s15 * y * z; G[12][1] = s15 * x * z; G[12][2] = s15 * x * y;
    G[13][0] = s58 * real(3) * (xx - yy); G[13][1] = s58 * real(-6) * x * y; G[13][2] = 0;
    G[14][0] = s58 * real(6) * x * y; G[14][1] = s58 * real(3) * (xx - yy); G[14][2] = 0;
    G[15][0] = x * (real(-6) * zz + real(1.5) * p2); G[15][1] = y * (real(-6) * zz + real(1.5) * p2);
    G[15][2] = z * (real(4) * zz - real(6) * p2);
    G[16][0] = s10q * z * (real(4) * zz - real(9) * xx - real(3) * yy); G[16][1] = s10q * real(-6) * x * y * z;
    G[16][2] = s10q * x * (real(12) * zz - real(3) * p2);
    G[17][0] = s10q * real(-6) * x * y * z; G[17][1] = s10q * z * (real(4) * zz - real(3) * xx - real(9) * yy);
    G[17][2] = s10q * y * (real(12) * zz - real(3) * p2);
    G[18][0] = s5 * x * (real(3) * zz - xx); G[18][1] = -s5 * y * (real(3) * zz - yy); G[18][2] = real(3) * s5 * z * (xx - yy);
    G[19][0] = s5h * y * (real(6) * zz - real(3) * xx - yy); G[19][1] = s5h * x * (real(6) * zz - xx - real(3) * yy);
    G[19][2] = real(6) * s5 * x * y * z;
    G[20][0] = s70q * real(3) * z * (xx - yy); G[20][1] = s70q * real(-6) * x * y * z; G[20][2] = s70q * x * (xx - real(3) * yy);
    G[21][0] = s70q * real(6) * x * y * z; G[21][1] = s70q * real(3) * z * (xx - yy); G[21][2] = s70q * y * (real(3) * xx - yy);
    G[22][0] = s35e * (real(4) * xx * x - real(12) * x * yy); G[22][1] = s35e * (real(4) * yy * y - real(12) * xx * y); G[22][2] = 0;
    G[23][0] = s35h * (real(3) * xx * y - yy * y); G[23][1] = s35h * (xx * x - real(3) * x * yy); G[23][2] = 0;
}

__host__ __device__ constexpr int l_of_lm(int lm) { return lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4; }

// one harmonic R_lm (same normalisation and order as harmonics()) and its
// gradient; with lm a compile-time constant only that polynomial is formed
template <int lm, typename real>
__device__ inline void harmonic_one(real x, real y, real z, real &Y, real &gx, real &gy, real &gz) {
    const real s3 = real(1.7320508075688772), s38 = real(0.61237243569579452),
               s15h = real(1.9364916731037085), s15 = real(3.8729833462074170),
               s58 = real(0.79056941504209483), s10q = real(0.79056941504209483),
               s5q = real(0.55901699437494742), s5 = real(2.2360679774997897), s5h = real(1.1180339887498949),
               s70q = real(2.0916500663351889), s35e = real(0.73950997288745200),
               s35h = real(2.9580398915498080);
    const real xx = x * x, yy = y * y, zz = z * z, p2 = xx + yy;
    if constexpr (lm == 0) { Y = x; gx = 1; gy = 0; gz = 0; }
    else if constexpr (lm == 1) { Y = y; gx = 0; gy = 1; gz = 0; }
    else if constexpr (lm == 2) { Y = z; gx = 0; gy = 0; gz = 1; }
    else if constexpr (lm == 3) { Y = s3 * x * y; gx = s3 * y; gy = s3 * x; gz = 0; }
    else if constexpr (lm == 4) { Y = s3 * y * z; gx = 0; gy = s3 * z; gz = s3 * y; }
    else if constexpr (lm == 5) { Y = real(0.5) * (real(2) * zz - p2); gx = -x; gy = -y; gz = real(2) * z; }
    else if constexpr (lm == 6) { Y = s3 * x * z; gx = s3 * z; gy = 0; gz = s3 * x; }
    else if constexpr (lm == 7) { Y = real(0.5) * s3 * (xx - yy); gx = s3 * x; gy = -s3 * y; gz = 0; }
    else if constexpr (lm == 8) {
        Y = z * (zz - real(1.5) * p2);
        gx = real(-3) * x * z; gy = real(-3) * y * z; gz = real(3) * zz - real(1.5) * p2;
    } else if constexpr (lm == 9) {
        Y = s38 * x * (real(4) * zz - p2);
        gx = s38 * (real(4) * zz - real(3) * xx - yy); gy = s38 * real(-2) * x * y; gz = s38 * real(8) * x * z;
    } else if constexpr (lm == 10) {
        Y = s38 * y * (real(4) * zz - p2);
        gx = s38 * real(-2) * x * y; gy = s38 * (real(4) * zz - xx - real(3) * yy); gz = s38 * real(8) * y * z;
    } else if constexpr (lm == 11) {
        Y = s15h * z * (xx - yy); gx = s15 * x * z; gy = -s15 * y * z; gz = s15h * (xx - yy);
    } else if constexpr (lm == 12) {
        Y = s15 * x * y * z; gx = s15 * y * z; gy = s15 * x * z; gz = s15 * x * y;
    } else if constexpr (lm == 13) {
        Y = s58 * x * (xx - real(3) * yy); gx = s58 * real(3) * (xx - yy); gy = s58 * real(-6) * x * y; gz = 0;
    } else if constexpr (lm == 14) {
        Y = s58 * y * (real(3) * xx - yy); gx = s58 * real(6) * x * y; gy = s58 * real(3) * (xx - yy); gz = 0;
    } else if constexpr (lm == 15) {
        Y = zz * zz - real(3) * zz * p2 + real(0.375) * p2 * p2;
        gx = x * (real(-6) * zz + real(1.5) * p2); gy = y * (real(-6) * zz + real(1.5) * p2);
        gz = z * (real(4) * zz - real(6) * p2);
    } else if constexpr (lm == 16) {
        Y = s10q * x * z * (real(4) * zz - real(3) * p2);
        gx = s10q * z * (real(4) * zz - real(9) * xx - real(3) * yy); gy = s10q * real(-6) * x * y * z;
        gz = s10q * x * (real(12) * zz - real(3) * p2);
    } else if constexpr (lm == 17) {
        Y = s10q * y * z * (real(4) * zz - real(3) * p2);
        gx = s10q * real(-6) * x * y * z; gy = s10q * z * (real(4) * zz - real(3) * xx - real(9) * yy);
        gz = s10q * y * (real(12) * zz - real(3) * p2);
    } else if constexpr (lm == 18) {
        Y = s5q * (xx - yy) * (real(6) * zz - p2);
        gx = s5 * x * (real(3) * zz - xx); gy = -s5 * y * (real(3) * zz - yy); gz = real(3) * s5 * z * (xx - yy);
    } else if constexpr (lm == 19) {
        Y = s5h * x * y * (real(6) * zz - p2);
        gx = s5h * y * (real(6) * zz - real(3) * xx - yy); gy = s5h * x * (real(6) * zz - xx - real(3) * yy);
        gz = real(6) * s5 * x * y * z;
    } else if constexpr (lm == 20) {
        Y = s70q * x * z * (xx - real(3) * yy);
        gx = s70q * real(3) * z * (xx - yy); gy = s70q * real(-6) * x * y * z; gz = s70q * x * (xx - real(3) * yy);
    } else if constexpr (lm == 21) {
        Y = s70q * y * z * (real(3) * xx - yy);
        gx = s70q * real(6) * x * y * z; gy = s70q * real(3) * z * (xx - yy); gz = s70q * y * (real(3) * xx - yy);
    } else if constexpr (lm == 22) {
        Y = s35e * (xx * xx - real(6) * xx * yy + yy * yy);
        gx = s35e * (real(4) * xx * x - real(12) * x * yy); gy = s35e * (real(4) * yy * y - real(12) * xx * y); gz = 0;
    } else {
        Y = s35h * x * y * (xx - yy);
        gx = s35h * (real(3) * xx * y - yy * y); gy = s35h * (xx * x - real(3) * x * yy); gz = 0;
    }
}

// the same with lm known only at run time (wave-uniform switch)
template <typename real>
__device__ inline void harmonic_dyn(int lm, real x, real y, real z, real &Y, real &gx, real &gy, real &gz) {
    switch (lm) {
#define NEP_HCASE(k) \
    case k: harmonic_one<k>(x, y, z, Y, gx, gy, gz); break;
        NEP_HCASE(0) NEP_HCASE(1) NEP_HCASE(2) NEP_HCASE(3) NEP_HCASE(4) NEP_HCASE(5) NEP_HCASE(6) NEP_HCASE(7)
        NEP_HCASE(8) NEP_HCASE(9) NEP_HCASE(10) NEP_HCASE(11) NEP_HCASE(12) NEP_HCASE(13) NEP_HCASE(14)
        NEP_HCASE(15) NEP_HCASE(16) NEP_HCASE(17) NEP_HCASE(18) NEP_HCASE(19) NEP_HCASE(20) NEP_HCASE(21)
        NEP_HCASE(22)
        default: harmonic_one<23>(x, y, z, Y, gx, gy, gz); break;
#undef NEP_HCASE
    }
}

// compile-time loop helper
template <int N, typename F>
__device__ inline void static_for(F &&f) {
    if constexpr (N > 0) {
        static_for<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the two 32x32->64
// multiplications and the Weyl key schedule.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// three standard normals for (seed, atom, step, stream) via Box-Muller on two
// Philox draws (x, y from draw 0, z = first normal of draw 1)
__device__ inline void gauss3(unsigned long long seed, uint32_t atom, unsigned long long step,
                              uint32_t stream, double xi[3]) {
    double z[3];
#pragma unroll
    for (uint32_t draw = 0; draw < 2; draw++) {
        uint32_t c[4] = {atom, (uint32_t)step, (uint32_t)(step >> 32), stream * 256u + draw};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const unsigned long long a = ((((unsigned long long)c[0]) << 32) | c[1]) >> 11;
        const unsigned long long b = ((((unsigned long long)c[2]) << 32) | c[3]) >> 11;
        const double u1 = 1.0 - (double)a * 0x1.0p-53;
        const double u2 = (double)b * 0x1.0p-53;
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 2.0 * PI * u2;
        if (draw == 0) {
            z[0] = rad * cos(ang);
            z[1] = rad * sin(ang);
        } else {
            z[2] = rad * cos(ang);
        }
    }
    xi[0] = z[0];
    xi[1] = z[1];
    xi[2] = z[2];
}

}  // namespace nep
