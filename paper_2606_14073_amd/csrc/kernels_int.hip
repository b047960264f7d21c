// kernels_int.hip -- the spin-lattice step on the device: velocity and
// position half-steps, the lattice Langevin step, the spin sweep over a fixed
// colouring of the spin carriers, and fixed-order per-replica reductions.
// Positions, velocities, spins and all sums are FP64.
#include "engine.h"

namespace nep {

namespace {

inline int nblk(int n, int b) { return (n + b - 1) / b; }

__global__ void k_kick(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const RepDev &R = S.rep[S.rid[i]];
    if (!R.active) return;
    const double c = 0.5 * R.dt * KAPPA / R.mass[i < S.N_fe ? 0 : 1];
    d4 v = S.vel[i];
    const d4 f = S.force[i];
    v.x += c * f.x;
    v.y += c * f.y;
    v.z += c * f.z;
    S.vel[i] = v;
}

__global__ void k_drift(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const RepDev &R = S.rep[S.rid[i]];
    if (!R.active) return;
    const double h = 0.5 * R.dt;
    d4 p = S.pos[i];
    const d4 v = S.vel[i];
    p.x += h * v.x;
    p.y += h * v.y;
    p.z += h * v.z;
    if (R.pbc[0]) p.x -= R.box[0] * floor(p.x / R.box[0]);
    if (R.pbc[1]) p.y -= R.box[1] * floor(p.y / R.box[1]);
    if (R.pbc[2]) p.z -= R.box[2] * floor(p.z / R.box[2]);
    S.pos[i] = p;
}

__device__ inline double temperature(const RepDev &R) { return R.T0 + (R.T1 - R.T0) * ramp_frac(R); }

__global__ void k_langevin(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const RepDev &R = S.rep[S.rid[i]];
    if (!R.active || R.ensemble != 1) return;
    const double c1 = exp(-R.gammaL * R.dt);
    const double sig = sqrt((1.0 - c1 * c1) * KAPPA * KB * temperature(R) / R.mass[i < S.N_fe ? 0 : 1]);
    double xi[3];
    gauss3(R.seed, (uint32_t)S.orig[i], (unsigned long long)R.step, 0u, xi);
    d4 v = S.vel[i];
    v.x = c1 * v.x + sig * xi[0];
    v.y = c1 * v.y + sig * xi[1];
    v.z = c1 * v.z + sig * xi[2];
    S.vel[i] = v;
}

// noise field of the step and the reference copies S^n, S_hat
__global__ void k_spin_prep(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    const RepDev &R = S.rep[S.rid[i]];
    if (!R.active) return;
    const double T = temperature(R);
    d4 e = {0, 0, 0, 0};
    if (!R.lsf && R.alpha > 0 && T > 0) {
        const double sig = sqrt(2.0 * R.alpha * KB * T * HBAR / R.dt);
        double xi[3];
        gauss3(R.seed, (uint32_t)S.orig[i], (unsigned long long)R.step, 1u, xi);
        e.x = sig * xi[0];
        e.y = sig * xi[1];
        e.z = sig * xi[2];
    }
    S.eta[i] = e;
    const d4 s = S.spin[i];
    S.spin_n[i] = s;
    S.spin_hat[i] = s;
}

// replicas whose self-consistent iteration has converged keep their spins
__device__ inline bool spin_pass_on(const RepDev &R) { return R.active && !R.sc_done; }

__global__ void k_spin_restore(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    if (!spin_pass_on(S.rep[S.rid[i]])) return;
    S.spin[i] = S.spin_n[i];
}

__global__ void k_spin_mid(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    if (!spin_pass_on(S.rep[S.rid[i]])) return;
    const d4 a = S.spin_n[i], b = S.spin[i];
    const double x = 0.5 * (a.x + b.x), y = 0.5 * (a.y + b.y), z = 0.5 * (a.z + b.z);
    // unit spins: the normalised average; spins of variable length: the average
    const double n = S.rep[S.rid[i]].lsf ? 1.0 : sqrt(x * x + y * y + z * z);
    d4 h = {x / n, y / n, z / n, 0.0};
    S.spin_hat[i] = h;
}

// sin(t) and 1 - cos(t) from their Taylor series (coefficients +-1/n!) through
// t^19 and t^20, for |t| <= 1 where the truncation error is below 1e-19; no
// cancellation in 1 - cos. Both are polynomials of degree 9 in u = t^2,
// evaluated in Estrin's form (pairs, then u^2, u^4, u^8): five dependent
// steps instead of nine, since the midpoint iteration is latency bound.
__device__ inline void sin_omc_taylor(double t, double &sn, double &omc) {
    const double u = t * t, u2 = u * u, u4 = u2 * u2, u8 = u4 * u4;
    // sin(t)/t = sum_k (-1)^k u^k / (2k+1)!
    const double s01 = fma(u, -1.0 / 6.0, 1.0);
    const double s23 = fma(u, -1.0 / 5040.0, 1.0 / 120.0);
    const double s45 = fma(u, -1.0 / 39916800.0, 1.0 / 362880.0);
    const double s67 = fma(u, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);
    const double s89 = fma(u, -1.0 / 121645100408832000.0, 1.0 / 355687428096000.0);
    const double ps = fma(u8, s89, fma(u4, fma(u2, s67, s45), fma(u2, s23, s01)));
    // (1 - cos t)/t^2 = sum_k (-1)^k u^k / (2k+2)!
    const double c01 = fma(u, -1.0 / 24.0, 0.5);
    const double c23 = fma(u, -1.0 / 40320.0, 1.0 / 720.0);
    const double c45 = fma(u, -1.0 / 479001600.0, 1.0 / 3628800.0);
    const double c67 = fma(u, -1.0 / 20922789888000.0, 1.0 / 87178291200.0);
    const double c89 = fma(u, -1.0 / 2432902008176640000.0, 1.0 / 6402373705728000.0);
    const double pc = fma(u8, c89, fma(u4, fma(u2, c67, c45), fma(u2, c23, c01)));
    sn = t * ps;
    omc = u * pc;
}

// 1/sqrt(x) for x > 0 in FP64: the hardware estimate y (relative error e0
// about 5e-8 on gfx950) refined by one third-order step,
// y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2, whose truncation error
// 5 e0^3 / 16 is far below rounding: the result is within 1 ulp.
__device__ inline double rsqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Value of lane K of this lane's quad (lanes 4q..4q+3), by DPP.
template <int K>
__device__ inline double quad_bcast(double v) {
    constexpr int ctrl = K | (K << 2) | (K << 4) | (K << 6);   // quad_perm [K, K, K, K]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// One coupling's contribution to the field on a spin: exchange J s_j, DMI
// D s_j x r, anisotropic exchange K (s_j . r) r, subtracted from h, with
// explicit fused multiply-adds and no other contraction.
__device__ inline void coupling_field(double J, double D, double K, double rx, double ry, double rz, double sx,
                                      double sy, double sz, double &hx, double &hy, double &hz) {
#pragma clang fp contract(off)
    const double sr = fma(sz, rz, fma(sy, ry, sx * rx));
    const double ks = K * sr;
    hx -= fma(J, sx, fma(D, fma(sy, rz, -(sz * ry)), ks * rx));
    hy -= fma(J, sy, fma(D, fma(sz, rx, -(sx * rz)), ks * ry));
    hz -= fma(J, sz, fma(D, fma(sx, ry, -(sy * rx)), ks * rz));
}

// One colour class: every spin takes an implicit-midpoint Rodrigues rotation
// over tau = dt/2 in the field of its (other-colour) neighbours, its own
// anisotropy/onsite terms at the midpoint, the Zeeman field and the noise.
// L lanes share a spin (L = 4, 8 or 16): they split the neighbour gather
// (couplings stored in colour-list order, so a wavefront reads contiguous
// records), reduce, and then solve the midpoint equation together (each quad
// of lanes evaluates the rotation at four points per Newton step); lane 0
// stores the result.
// The field sum has one order whatever L is: sixteen virtual lanes v each
// add the couplings in slots v, v + 16, v + 32, ... in turn, and a butterfly
// over v (xor 1, 2, 4, 8) adds the sixteen partial sums. Lane l of L carries
// the virtual lanes l + L k, k < 16 / L; the butterfly levels below L run
// across lanes and the others inside the lane. A spin's result thus has the
// same bits with any L, so each launch takes the L that suits the size of
// its colour class (fewer, fuller waves for large classes, more workgroups
// for small ones) and a replica still gives the same bits alone and in any
// batch.
// Latency is what bounds a colour class, so the loads are issued in two
// waves: everything indexed by the colour-list position (atom, replica,
// coupling count, self terms, the first 32 coupling slots, read whether or
// not they are in use and masked afterwards), then the neighbours' spins, the
// spin itself, its noise and the replica record.
constexpr int SWEEP_V = 16;              // virtual lanes of the field sum
constexpr int SWEEP_WIDE_MIN = 8192;     // classes of at least this many spins take 8 lanes per spin
constexpr int SWEEP_WIDER_MIN = 32768;   // and of at least this many 4

// turns = 2 takes the colour twice in a row (the end of the ascending and the
// start of the descending pass): the neighbour field is the same for both
// rotations, the second starts from the first one's result.
// The kernel's own arithmetic is not contracted: the compiler would fuse
// multiplies and adds differently in the two lane layouts (their code is
// scheduled apart), and their results would then differ in the last bit;
// where a fused multiply-add is wanted it is written out.
template <typename real, int L>
__global__ void __launch_bounds__(256) k_sweep(Sys S, Work<real> W, int base, int count, int turns, int visit0) {
#pragma clang fp contract(off)
    constexpr int P = SWEEP_V / L;   // virtual lanes per lane
    constexpr int R0 = 2 * P;        // coupling slots per lane loaded up front
    const int lane = threadIdx.x & (L - 1);
    const int t = blockIdx.x * (256 / L) + threadIdx.x / L;
    if (t >= count) return;
    const int p = base + t;
    const size_t lf = S.N_fe;
    // first wave of loads; up-front slot u = 2 k + w is slot lane + L k + 16 w
    const int i = S.col_idx[p];
    const int r = S.col_rid[p];
    const int nc = W.cpl_n[p];
    const real *o = W.selfc + (size_t)p * 8;
    const double Axx = o[0], Ayy = o[1], Azz = o[2], Axy = o[3], Axz = o[4], Ayz = o[5], os = o[6];
    int cj[R0];
    double cv[R0][6];
#pragma unroll
    for (int u = 0; u < R0; u++) {
        const size_t q = (size_t)(lane + L * (u >> 1) + SWEEP_V * (u & 1)) * lf + p;
        cj[u] = W.cpl_j[q];
        const real *c = W.cpl + q * 6;
#pragma unroll
        for (int x = 0; x < 6; x++) cv[u][x] = c[x];
    }
    // second wave
    const RepDev &R = S.rep[r];
    const d4 e = S.eta[i];
    const d4 s4 = S.spin[i];
    double px[P], py[P], pz[P];
#pragma unroll
    for (int k = 0; k < P; k++) px[k] = py[k] = pz[k] = 0;
    d4 sj[R0];
#pragma unroll
    for (int u = 0; u < R0; u++) sj[u] = S.spin[lane + L * (u >> 1) + SWEEP_V * (u & 1) < nc ? cj[u] : i];
#pragma unroll
    for (int u = 0; u < R0; u++) {
        const int k = u >> 1;
        if (lane + L * k + SWEEP_V * (u & 1) >= nc) continue;
        coupling_field(cv[u][0], cv[u][1], cv[u][2], cv[u][3], cv[u][4], cv[u][5], sj[u].x, sj[u].y, sj[u].z, px[k],
                       py[k], pz[k]);
    }
    // spins with more than 32 couplings
#pragma unroll
    for (int k = 0; k < P; k++)
        for (int s = lane + L * k + 2 * SWEEP_V; s < nc; s += SWEEP_V) {
            const int j = W.cpl_j[(size_t)s * lf + p];
            const real *c = W.cpl + ((size_t)s * lf + p) * 6;
            const d4 v = S.spin[j];
            coupling_field(c[0], c[1], c[2], c[3], c[4], c[5], v.x, v.y, v.z, px[k], py[k], pz[k]);
        }
    // butterfly: levels 1 .. L/2 across the lanes, then L .. 8 inside them
#pragma unroll
    for (int m = 1; m < L; m <<= 1)
#pragma unroll
        for (int k = 0; k < P; k++) {
            px[k] += __shfl_xor(px[k], m);
            py[k] += __shfl_xor(py[k], m);
            pz[k] += __shfl_xor(pz[k], m);
        }
#pragma unroll
    for (int b = 1; b < P; b <<= 1)
#pragma unroll
        for (int k = 0; k < P; k += 2 * b) {
            px[k] += px[k + b];
            py[k] += py[k + b];
            pz[k] += pz[k + b];
        }
    double hx = px[0], hy = py[0], hz = pz[0];
    if (!spin_pass_on(R)) return;
    const double fr = ramp_frac(R), zs = R.mu_s * MUB;
    hx += fma(zs, fma(R.B1[0] - R.B0[0], fr, R.B0[0]), e.x);
    hy += fma(zs, fma(R.B1[1] - R.B0[1], fr, R.B0[1]), e.y);
    hz += fma(zs, fma(R.B1[2] - R.B0[2], fr, R.B0[2]), e.z);
    const double al = R.alpha, inv = 1.0 / fma(al, al, 1.0), tau = 0.5 * R.dt / HBAR;
    const double tol = R.mid_tol;
    const int cap = R.mid_cap;
    const double Dxx = Axx + os, Dyy = Ayy + os, Dzz = Azz + os;   // A_i + o_i I
    const double la2 = 2.0 * R.landau_a, lb4 = 4.0 * R.landau_b;   // onsite moment-length term
    double sx = s4.x, sy = s4.y, sz = s4.z;
    double len = 1.0;    // length of the midpoint vector: 1, or |s| for spins of variable length
    // G(y): the spin rotated about the precession vector taken at the
    // midpoint m = len (s + y)/|s + y| (field, damping, anisotropy, onsite
    // and moment-length terms evaluated at m), by the angle |w| tau (Rodrigues)
    auto rotate = [&](double px, double py, double pz, double &nx, double &ny, double &nz) {
        double mx = sx + px, my = sy + py, mz = sz + pz;
        const double mn = rsqrt_nr(fma(mz, mz, fma(my, my, mx * mx))) * len;
        mx *= mn;
        my *= mn;
        mz *= mn;
        const double kl = fma(lb4, fma(mz, mz, fma(my, my, mx * mx)), la2);
        const double h0 = fma(-kl, mx, fma(-2.0, fma(Axz, mz, fma(Axy, my, Dxx * mx)), hx));
        const double h1 = fma(-kl, my, fma(-2.0, fma(Ayz, mz, fma(Dyy, my, Axy * mx)), hy));
        const double h2 = fma(-kl, mz, fma(-2.0, fma(Dzz, mz, fma(Ayz, my, Axz * mx)), hz));
        const double wx = fma(al, fma(my, h2, -(mz * h1)), h0) * inv;
        const double wy = fma(al, fma(mz, h0, -(mx * h2)), h1) * inv;
        const double wz = fma(al, fma(mx, h1, -(my * h0)), h2) * inv;
        const double w2 = fma(wz, wz, fma(wy, wy, wx * wx));
        if (w2 == 0.0) {
            nx = sx;
            ny = sy;
            nz = sz;
            return;
        }
        const double iw = rsqrt_nr(w2);
        const double th = w2 * iw * tau, ath = fabs(th);   // negative for a backward step
        double sn, cs, omc;
        if (ath <= 1.0) {
            sin_omc_taylor(th, sn, omc);
            cs = 1.0 - omc;
        } else {
            sincos(th, &sn, &cs);
            omc = 1.0 - cs;
        }
        const double ux = wx * iw, uy = wy * iw, uz = wz * iw;
        const double us = fma(uz, sz, fma(uy, sy, ux * sx)), uo = us * omc;
        nx = fma(ux, uo, fma(fma(uy, sz, -(uz * sy)), sn, sx * cs));
        ny = fma(uy, uo, fma(fma(uz, sx, -(ux * sz)), sn, sy * cs));
        nz = fma(uz, uo, fma(fma(ux, sy, -(uy * sx)), sn, sz * cs));
    };
    // The midpoint equation y = G(y) is solved by Newton's method on
    // G(y) - y with a forward-difference Jacobian: the four lanes of each
    // quad evaluate G at y and at y + h e_x, y + h e_y, y + h e_z at once
    // (the spin's other lanes are otherwise idle here), exchange the results by
    // quad broadcasts and take the same step. The iteration stops, as the
    // plain fixed-point one, when |G(y) - y| <= tol, and returns G(y): a
    // rotation of the spin, so its length is kept. The Jacobian's relative
    // error (about 1e-8 from the step h = 2^-26) only slows the final
    // convergence to linear with that ratio.
    const int sub = lane & 3;
    constexpr double FD_H = 0x1p-26, FD_IH = 0x1p26;
    // Spins of variable length with damping: the rotation sits between two
    // longitudinal half steps of the Langevin dynamics over dt/4 each,
    // x += (gamma t/hbar) h(x) + sqrt(2 gamma kB T t/hbar) xi, h the full
    // field at x (neighbours, Zeeman, anisotropy, onsite and moment-length
    // terms), xi the Philox normals of streams 2 + 2 visit and 3 + 2 visit
    // (visit 0 ascending, 1 descending); every lane of the spin takes them
    // alike.
    const bool lsf = R.lsf != 0, lsf_damp = lsf && R.lsf_gamma > 0;
    const double T = lsf_damp ? temperature(R) : 0.0;
    auto lsf_half = [&](double &x, double &y, double &z, uint32_t stream) {
        const double t = 0.25 * R.dt;
        const double kl = la2 + lb4 * (x * x + y * y + z * z);
        const double f0 = hx - 2.0 * (Dxx * x + Axy * y + Axz * z) - kl * x;
        const double f1 = hy - 2.0 * (Axy * x + Dyy * y + Ayz * z) - kl * y;
        const double f2 = hz - 2.0 * (Axz * x + Ayz * y + Dzz * z) - kl * z;
        double xi[3] = {0.0, 0.0, 0.0};
        if (T > 0) gauss3(R.seed, (uint32_t)S.orig[i], (unsigned long long)R.step, stream, xi);
        const double k = R.lsf_gamma * t / HBAR, sig = sqrt(2.0 * R.lsf_gamma * KB * T * t / HBAR);
        x += k * f0 + sig * xi[0];
        y += k * f1 + sig * xi[1];
        z += k * f2 + sig * xi[2];
    };
    double yx = sx, yy = sy, yz = sz;
    int ncapped = 0;
    for (int turn = 0; turn < turns; turn++) {
        if (turn) {
            sx = yx;
            sy = yy;
            sz = yz;
        }
        const uint32_t visit = (uint32_t)(visit0 + turn);
        if (lsf_damp) lsf_half(sx, sy, sz, 2u + 2u * visit);
        if (lsf) len = sqrt(sx * sx + sy * sy + sz * sz);
        yx = sx;
        yy = sy;
        yz = sz;
        for (int it = 0; it < cap; it++) {
            double nx, ny, nz;
            rotate(yx + (sub == 1 ? FD_H : 0.0), yy + (sub == 2 ? FD_H : 0.0), yz + (sub == 3 ? FD_H : 0.0), nx, ny,
                   nz);
            const double g0x = quad_bcast<0>(nx), g0y = quad_bcast<0>(ny), g0z = quad_bcast<0>(nz);
            const double rx = g0x - yx, ry = g0y - yy, rz = g0z - yz;
            const double diff = fmax(fabs(rx), fmax(fabs(ry), fabs(rz)));
            if (diff <= tol || it + 1 == cap) {
                yx = g0x;
                yy = g0y;
                yz = g0z;
                ncapped += diff > tol;
                break;
            }
            // A = I - J, J columns (G(y + h e_c) - G(y)) / h
            const double a00 = 1.0 - (quad_bcast<1>(nx) - g0x) * FD_IH, a10 = -(quad_bcast<1>(ny) - g0y) * FD_IH,
                         a20 = -(quad_bcast<1>(nz) - g0z) * FD_IH;
            const double a01 = -(quad_bcast<2>(nx) - g0x) * FD_IH, a11 = 1.0 - (quad_bcast<2>(ny) - g0y) * FD_IH,
                         a21 = -(quad_bcast<2>(nz) - g0z) * FD_IH;
            const double a02 = -(quad_bcast<3>(nx) - g0x) * FD_IH, a12 = -(quad_bcast<3>(ny) - g0y) * FD_IH,
                         a22 = 1.0 - (quad_bcast<3>(nz) - g0z) * FD_IH;
            // y += A^-1 r (Cramer's rule); a plain fixed-point step if A is not
            // safely invertible (never for a contracting map)
            auto det2 = [](double a, double b, double c, double d) { return fma(a, b, -(c * d)); };   // ab - cd
            const double c00 = det2(a11, a22, a12, a21), c01 = det2(a12, a20, a10, a22), c02 = det2(a10, a21, a11, a20);
            const double det = fma(a02, c02, fma(a01, c01, a00 * c00));
            if (fabs(det) > 0.25) {
                const double id = 1.0 / det;
                yx += fma(det2(a01, a12, a02, a11), rz, fma(det2(a02, a21, a01, a22), ry, c00 * rx)) * id;
                yy += fma(det2(a02, a10, a00, a12), rz, fma(det2(a00, a22, a02, a20), ry, c01 * rx)) * id;
                yz += fma(det2(a00, a11, a01, a10), rz, fma(det2(a01, a20, a00, a21), ry, c02 * rx)) * id;
            } else {
                yx = g0x;
                yy = g0y;
                yz = g0z;
            }
        }
        if (lsf_damp) lsf_half(yx, yy, yz, 3u + 2u * visit);
    }
    if (lane == 0) {
        d4 out = {yx, yy, yz, 0.0};
        S.spin[i] = out;
        if (ncapped) atomicAdd(&S.rep[r].capped, ncapped);
    }
}

// Re-layout of the resident replicas: atom k of the new layout takes the state
// rows of atom src[k] of the old one, whose five arrays were copied whole to
// the staging buffer; src[k] = -1 marks atoms of replicas new to the device.
__global__ void __launch_bounds__(256) k_gather_state(const d4 *stage, size_t n_old, const int *src, int n, d4 *pos,
                                                      d4 *vel, d4 *spin, d4 *force, d4 *field) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int s = src[k];
    if (s < 0 || (size_t)s >= n_old) return;
    pos[k] = stage[s];
    vel[k] = stage[n_old + s];
    spin[k] = stage[2 * n_old + s];
    force[k] = stage[3 * n_old + s];
    field[k] = stage[4 * n_old + s];
}

__global__ void k_set_active(RepDev *rep, const int *act, int n) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n && act[r] >= 0) rep[r].active = act[r];
}

__global__ void k_step_end(Sys S) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= S.n_rep) return;
    RepDev &R = S.rep[r];
    if (!R.active) return;
    if (R.failed & 3) {      // list overflow or coupled same-colour spins: the step is void
        R.active = 0;
        return;
    }
    R.step += 1;
    R.sc_done = 0;
    R.capped = 0;
    // a replica waiting for a new colouring stops after this (exact) step
    if (R.step >= R.step_end || (R.failed & 4)) R.active = 0;
}

// Self-consistent midpoint (Sec. 5.1): the corrector is a fixed-point
// iteration x -> g(x) on the end-of-step spins, g being the sweep at the
// midpoint normalise((S^n + x)/2); x^(0) = S^n. After each sweep, per spin
// carrier of an iterating replica: the residual f = g - x and its max norm
// (non-negative doubles order like their bit patterns, so an integer max over
// the bits is the max; a wave reduces first and issues one atomic when all its
// lanes belong to one replica). Plain iteration keeps x = g for the next pass.
// The accelerated variant (depth > 0, one replica) stores the differences
// dF = f - f_prev, dG = g - g_prev in a ring of depth slots and sums, per
// workgroup in a fixed order, the Gram entries dF_a . dF_b and dF_a . f of
// the mk newest columns.
__device__ inline int sc_slot(int pass, int age, int depth) {   // ring slot of the column made `age` passes ago
    return ((pass - 1 - age) % depth + depth) % depth;
}

__global__ void __launch_bounds__(256) k_sc_check(Sys S, int pass, int depth, int mk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int r = -1;
    double d = 0;
    double3 f = {0, 0, 0};
    bool on = false;
    const size_t lf = S.N_fe;
    if (i < S.N_fe) {
        const int ri = S.rid[i];
        const RepDev &R = S.rep[ri];
        if (spin_pass_on(R) && R.sc_tol > 0) {
            on = true;
            const d4 g = S.spin[i];
            const d4 x = pass == 0 ? S.spin_n[i] : S.sc_x[i];
            f = make_double3(g.x - x.x, g.y - x.y, g.z - x.z);
            d = fmax(fabs(f.x), fmax(fabs(f.y), fabs(f.z)));
            r = pass > 0 ? ri : -1;
            if (depth == 0) {
                S.sc_x[i] = g;
            } else {
                if (pass > 0) {
                    const int sl = sc_slot(pass, 0, depth);
                    const d4 fp = S.sc_f[i], gp = S.sc_g[i];
                    S.sc_dF[sl * lf + i] = d4{f.x - fp.x, f.y - fp.y, f.z - fp.z, 0.0};
                    S.sc_dG[sl * lf + i] = d4{g.x - gp.x, g.y - gp.y, g.z - gp.z, 0.0};
                }
                S.sc_f[i] = d4{f.x, f.y, f.z, 0.0};
                S.sc_g[i] = g;
            }
        }
    }
    const int r0 = __shfl(r, 0);
    if (__all(r == r0)) {
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) d = fmax(d, __shfl_xor(d, m));
        if ((threadIdx.x & 63) == 0 && r0 >= 0)
            atomicMax(&S.rep[r0].sc_delta, (unsigned long long)__double_as_longlong(d));
    } else if (r >= 0) {
        atomicMax(&S.rep[r].sc_delta, (unsigned long long)__double_as_longlong(d));
    }
    if (mk == 0) return;   // uniform over the grid
    // Gram entries of the mk newest columns (age order), this workgroup's atoms
    __shared__ double red[4][SC_NK];
    double3 c[SC_MAXD];
#pragma unroll
    for (int a = 0; a < SC_MAXD; a++) {
        c[a] = make_double3(0, 0, 0);
        if (a < mk && on) {
            const d4 v = S.sc_dF[sc_slot(pass, a, depth) * lf + i];
            c[a] = make_double3(v.x, v.y, v.z);
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int k = 0;
#pragma unroll
    for (int a = 0; a < SC_MAXD; a++) {
        if (a >= mk) break;
#pragma unroll
        for (int b = 0; b <= a; b++) {
            double v = c[a].x * c[b].x + c[a].y * c[b].y + c[a].z * c[b].z;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
            if (lane == 0) red[wv][k] = v;
            k++;
        }
        double v = c[a].x * f.x + c[a].y * f.y + c[a].z * f.z;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
        if (lane == 0) red[wv][k] = v;
        k++;
    }
    __syncthreads();
    const int nk = mk * (mk + 1) / 2 + mk;
    if (threadIdx.x < nk) {
        const int t = threadIdx.x;
        S.sc_part[(size_t)blockIdx.x * SC_NK + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
}

// One workgroup: converged or capped replicas stop; count the others. A
// replica with a fixed number of correctors (sc_tol 0) iterating beside
// others stops after its k_corr corrector passes, as it would alone; every
// replica records its pass count and last change when it stops. With
// mixing, the Gram matrix is summed over the workgroups in order and the
// regularised normal equations (G + lam I) gam = r, lam = reg * trace(G) / mk,
// are solved by Cholesky; a pivot below 1e-13 of its diagonal entry (a column
// in the span of the others) gives the plain step. sc_out: pending replicas,
// largest change of this pass, used columns, gam[mk].
__global__ void __launch_bounds__(256) k_sc_decide(Sys S, int pass, int mk, int nblocks, double reg, int k_corr) {
    __shared__ int cnt;
    __shared__ unsigned long long dmax;
    __shared__ double sum[SC_NK];
    if (threadIdx.x == 0) {
        cnt = 0;
        dmax = 0;
    }
    __syncthreads();
    int mine = 0;
    for (int r = threadIdx.x; r < S.n_rep; r += blockDim.x) {
        RepDev &R = S.rep[r];
        if (!R.active || R.sc_done) continue;
        if (R.sc_tol <= 0) {
            if (pass >= k_corr) {
                R.sc_done = 1;
                R.sc_passes = pass + 1;
                R.sc_last = 0;
            } else {
                mine++;
            }
            continue;
        }
        const double dl = __longlong_as_double((long long)R.sc_delta);
        if (pass >= 1) atomicMax(&dmax, R.sc_delta);
        if (pass >= 1 && (dl <= R.sc_tol || pass >= R.sc_max)) {
            R.sc_done = 1;
            R.sc_passes = pass + 1;
            R.sc_last = dl;
        }
        R.sc_delta = 0;
        mine += !R.sc_done;
    }
    if (mine) atomicAdd(&cnt, mine);
    const int nk = mk * (mk + 1) / 2 + mk;
    if (threadIdx.x < nk) {
        double v = 0;
        for (int b = 0; b < nblocks; b++) v += S.sc_part[(size_t)b * SC_NK + threadIdx.x];
        sum[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double *out = S.sc_out;
    out[0] = cnt;
    out[1] = __longlong_as_double((long long)dmax);
    out[2] = 0;
    if (mk == 0 || cnt == 0) return;
    double G[SC_MAXD][SC_MAXD], rh[SC_MAXD], L[SC_MAXD][SC_MAXD], y[SC_MAXD], gam[SC_MAXD];
    int k = 0;
    for (int a = 0; a < mk; a++) {
        for (int b = 0; b <= a; b++) G[a][b] = G[b][a] = sum[k++];
        rh[a] = sum[k++];
    }
    double tr = 0;
    for (int a = 0; a < mk; a++) tr += G[a][a];
    if (!(tr > 0)) return;
    const double lam = reg * tr / mk;
    for (int a = 0; a < mk; a++) {
        for (int b = 0; b <= a; b++) {
            double v = G[a][b] + (a == b ? lam : 0.0);
            for (int c = 0; c < b; c++) v -= L[a][c] * L[b][c];
            if (a == b) {
                if (!(v > 1e-13 * (G[a][a] + lam))) return;
                L[a][a] = sqrt(v);
            } else {
                L[a][b] = v / L[b][b];
            }
        }
    }
    for (int a = 0; a < mk; a++) {
        double v = rh[a];
        for (int c = 0; c < a; c++) v -= L[a][c] * y[c];
        y[a] = v / L[a][a];
    }
    for (int a = mk - 1; a >= 0; a--) {
        double v = y[a];
        for (int c = a + 1; c < mk; c++) v -= L[c][a] * gam[c];
        gam[a] = v / L[a][a];
    }
    for (int a = 0; a < mk; a++) out[3 + a] = gam[a];
    out[2] = mk;
}

// mixed iterate x = g - sum_a gam_a dG_a (the plain x = g when no columns are
// used) and the midpoint spins normalise((S^n + x)/2) of the next pass
__global__ void __launch_bounds__(256) k_sc_mix(Sys S, int pass, int depth) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    if (!spin_pass_on(S.rep[S.rid[i]])) return;
    const size_t lf = S.N_fe;
    const int used = (int)S.sc_out[2];
    const d4 g = S.spin[i];
    double x = g.x, y = g.y, z = g.z;
    for (int a = 0; a < used; a++) {
        const double ga = S.sc_out[3 + a];
        const d4 v = S.sc_dG[sc_slot(pass, a, depth) * lf + i];
        x -= ga * v.x;
        y -= ga * v.y;
        z -= ga * v.z;
    }
    S.sc_x[i] = d4{x, y, z, 0.0};
    const d4 a = S.spin_n[i];
    const double mx = 0.5 * (a.x + x), my = 0.5 * (a.y + y), mz = 0.5 * (a.z + z);
    const double n = S.rep[S.rid[i]].lsf ? 1.0 : sqrt(mx * mx + my * my + mz * mz);
    S.spin_hat[i] = d4{mx / n, my / n, mz / n, 0.0};
}

// per-chunk partial sums of the observables (fixed tree), then per replica
template <typename real>
__global__ void __launch_bounds__(256) k_obs_partial(Sys S, Work<real> W, const Chunk *chunks, double *partial) {
    __shared__ double red[NOBS][256];
    const Chunk c = chunks[blockIdx.x];
    const int t = threadIdx.x;
    double v[NOBS];
#pragma unroll
    for (int k = 0; k < NOBS; k++) v[k] = 0;
    const int i = c.begin + t;
    if (i < c.end) {
        const RepDev &R = S.rep[c.rid];
        const int fe = i < S.N_fe;
        const d4 vel = S.vel[i], s = S.spin[i], H = S.field[i], p = S.pos[i], F = S.force[i];
        const double m = R.mass[fe ? 0 : 1];
        v[0] = (double)W.Ei[i];
        v[1] = 0.5 * m * (vel.x * vel.x + vel.y * vel.y + vel.z * vel.z) / KAPPA;
        if (fe) {
            const double fr = ramp_frac(R), zs = R.mu_s * MUB;
            v[2] = -zs * ((R.B0[0] + (R.B1[0] - R.B0[0]) * fr) * s.x + (R.B0[1] + (R.B1[1] - R.B0[1]) * fr) * s.y +
                          (R.B0[2] + (R.B1[2] - R.B0[2]) * fr) * s.z);
            const double cx = s.y * H.z - s.z * H.y, cy = s.z * H.x - s.x * H.z, cz = s.x * H.y - s.y * H.x;
            v[3] = cx * cx + cy * cy + cz * cz;
            v[4] = s.x * H.x + s.y * H.y + s.z * H.z;
            v[5] = s.x;
            v[6] = s.y;
            v[7] = s.z;
            v[8] = sqrt(s.x * s.x + s.y * s.y + s.z * s.z);
        }
        const double chk = p.x + p.y + p.z + vel.x + vel.y + vel.z + s.x + s.y + s.z + F.x + F.y + F.z + v[0];
        v[NOBS - 1] = isfinite(chk) ? 0.0 : 1.0;
    }
#pragma unroll
    for (int k = 0; k < NOBS; k++) red[k][t] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int k = 0; k < NOBS; k++) red[k][t] += red[k][t + off];
        __syncthreads();
    }
    if (t < NOBS) partial[(size_t)blockIdx.x * NOBS + t] = red[t][0];
}

// one workgroup per replica: thread t sums chunks t, t+256, ... in order,
// then a fixed tree; the result depends only on the replica's own chunks
__global__ void __launch_bounds__(256) k_obs_final(Sys S, const int *chunk_ptr, const double *partial, double *out) {
    __shared__ double red[NOBS][256];
    const int r = blockIdx.x, t = threadIdx.x;
    double v[NOBS];
#pragma unroll
    for (int k = 0; k < NOBS; k++) v[k] = 0;
    for (int c = chunk_ptr[r] + t; c < chunk_ptr[r + 1]; c += 256)
#pragma unroll
        for (int k = 0; k < NOBS; k++) v[k] += partial[(size_t)c * NOBS + k];
#pragma unroll
    for (int k = 0; k < NOBS; k++) red[k][t] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int k = 0; k < NOBS; k++) red[k][t] += red[k][t + off];
        __syncthreads();
    }
    // slot 9: the replica's capped rotations (a counter, not a sum); slot
    // NOBS-1 counts non-finite atoms
    if (t < NOBS) out[(size_t)r * NOBS + t] = t == 9 ? (double)S.rep[r].capped : red[t][0];
}

}  // namespace

void launch_kick(const Sys &S, hipStream_t st) {
    if (S.N) hipLaunchKernelGGL(k_kick, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
}
void launch_drift(const Sys &S, hipStream_t st) {
    if (S.N) hipLaunchKernelGGL(k_drift, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
}
void launch_langevin(const Sys &S, hipStream_t st) {
    if (S.N) hipLaunchKernelGGL(k_langevin, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
}
void launch_spin_prep(const Sys &S, hipStream_t st) {
    if (S.N_fe) hipLaunchKernelGGL(k_spin_prep, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S);
}
void launch_spin_restore(const Sys &S, hipStream_t st) {
    if (S.N_fe) hipLaunchKernelGGL(k_spin_restore, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S);
}
void launch_spin_mid(const Sys &S, hipStream_t st) {
    if (S.N_fe) hipLaunchKernelGGL(k_spin_mid, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S);
}
void launch_step_end(const Sys &S, hipStream_t st) {
    if (S.n_rep) hipLaunchKernelGGL(k_step_end, dim3(nblk(S.n_rep, 64)), dim3(64), 0, st, S);
}
void launch_set_active(RepDev *rep, const int *act, int n, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_set_active, dim3(nblk(n, 64)), dim3(64), 0, st, rep, act, n);
}
void launch_gather_state(const d4 *stage, size_t n_old, const int *src, int n, d4 *pos, d4 *vel, d4 *spin, d4 *force,
                         d4 *field, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_gather_state, dim3(nblk(n, 256)), dim3(256), 0, st, stage, n_old, src, n, pos, vel,
                              spin, force, field);
}
int sc_part_blocks(int n_fe) { return nblk(n_fe, 256); }
void launch_sc_check(const Sys &S, int pass, int depth, double reg, int k_corr, hipStream_t st) {
    const int mk = depth > 0 ? (pass < depth ? pass : depth) : 0;
    const int nb = nblk(S.N_fe, 256);
    if (S.N_fe) hipLaunchKernelGGL(k_sc_check, dim3(nb), dim3(256), 0, st, S, pass, depth, mk);
    hipLaunchKernelGGL(k_sc_decide, dim3(1), dim3(256), 0, st, S, pass, S.N_fe ? mk : 0, nb, reg, k_corr);
}
void launch_sc_mix(const Sys &S, int pass, int depth, hipStream_t st) {
    if (S.N_fe) hipLaunchKernelGGL(k_sc_mix, dim3(nblk(S.N_fe, 256)), dim3(256), 0, st, S, pass, depth);
}

// colours 0, 1, .., C-1 and then C-1, .., 0; the two visits of colour C-1 are
// one launch
template <typename real>
void launch_sweep(const Sys &S, const Work<real> &W, const int *col_ptr_host, int n_colours, hipStream_t st) {
    for (int pass = 0; pass < 2; pass++)
        for (int cc = 0; cc < n_colours; cc++) {
            if (pass == 1 && cc == 0) continue;       // done as the second turn of the last ascending launch
            const int c = pass == 0 ? cc : n_colours - 1 - cc;
            const int turns = (pass == 0 && cc == n_colours - 1) ? 2 : 1;
            const int b = col_ptr_host[c], n = col_ptr_host[c + 1] - b;
            if (n >= SWEEP_WIDER_MIN)
                hipLaunchKernelGGL((k_sweep<real, 4>), dim3(nblk(n, 256 / 4)), dim3(256), 0, st, S, W, b, n, turns,
                                   pass);
            else if (n >= SWEEP_WIDE_MIN)
                hipLaunchKernelGGL((k_sweep<real, 8>), dim3(nblk(n, 256 / 8)), dim3(256), 0, st, S, W, b, n, turns,
                                   pass);
            else if (n > 0)
                hipLaunchKernelGGL((k_sweep<real, 16>), dim3(nblk(n, 256 / 16)), dim3(256), 0, st, S, W, b, n, turns,
                                   pass);
        }
}

template <typename real>
void launch_observe(const Sys &S, const Work<real> &W, const Chunk *chunks, int n_chunks,
                    const int *chunk_ptr, double *partial, double *out, hipStream_t st) {
    if (n_chunks == 0) return;
    hipLaunchKernelGGL(k_obs_partial<real>, dim3(n_chunks), dim3(256), 0, st, S, W, chunks, partial);
    hipLaunchKernelGGL(k_obs_final, dim3(S.n_rep), dim3(256), 0, st, S, chunk_ptr, partial, out);
}

template void launch_sweep<double>(const Sys &, const Work<double> &, const int *, int, hipStream_t);
template void launch_sweep<float>(const Sys &, const Work<float> &, const int *, int, hipStream_t);
template void launch_observe<double>(const Sys &, const Work<double> &, const Chunk *, int, const int *, double *,
                                     double *, hipStream_t);
template void launch_observe<float>(const Sys &, const Work<float> &, const Chunk *, int, const int *, double *,
                                    double *, hipStream_t);

}  // namespace nep
