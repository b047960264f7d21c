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
    const double c = 0.5 * R.dt * KAPPA / mass_of(i < S.N_fe ? 0 : 1);
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
    const double sig = sqrt((1.0 - c1 * c1) * KAPPA * KB * temperature(R) / mass_of(i < S.N_fe ? 0 : 1));
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
    if (R.alpha > 0 && T > 0) {
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

__global__ void k_spin_restore(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    if (!S.rep[S.rid[i]].active) return;
    S.spin[i] = S.spin_n[i];
}

__global__ void k_spin_mid(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N_fe) return;
    if (!S.rep[S.rid[i]].active) return;
    const d4 a = S.spin_n[i], b = S.spin[i];
    const double x = 0.5 * (a.x + b.x), y = 0.5 * (a.y + b.y), z = 0.5 * (a.z + b.z);
    const double n = sqrt(x * x + y * y + z * z);
    d4 h = {x / n, y / n, z / n, 0.0};
    S.spin_hat[i] = h;
}

// sin(t) and 1 - cos(t) from their Taylor series (coefficients +-1/n!), for
// |t| <= 1 where the truncation error is below 1e-19; no cancellation in 1 - cos.
__device__ inline void sin_omc_taylor(double t, double &sn, double &omc) {
    const double t2 = t * t;
    double ps = 1.0 / 121645100408832000.0;              // 1/19!
    ps = ps * -t2 + 1.0 / 355687428096000.0;             // 1/17!
    ps = ps * -t2 + 1.0 / 1307674368000.0;               // 1/15!
    ps = ps * -t2 + 1.0 / 6227020800.0;                  // 1/13!
    ps = ps * -t2 + 1.0 / 39916800.0;                    // 1/11!
    ps = ps * -t2 + 1.0 / 362880.0;                      // 1/9!
    ps = ps * -t2 + 1.0 / 5040.0;                        // 1/7!
    ps = ps * -t2 + 1.0 / 120.0;                         // 1/5!
    ps = ps * -t2 + 1.0 / 6.0;                           // 1/3!
    ps = ps * -t2 + 1.0;
    sn = t * ps;
    double pc = 1.0 / 2432902008176640000.0;             // 1/20!
    pc = pc * -t2 + 1.0 / 6402373705728000.0;            // 1/18!
    pc = pc * -t2 + 1.0 / 20922789888000.0;              // 1/16!
    pc = pc * -t2 + 1.0 / 87178291200.0;                 // 1/14!
    pc = pc * -t2 + 1.0 / 479001600.0;                   // 1/12!
    pc = pc * -t2 + 1.0 / 3628800.0;                     // 1/10!
    pc = pc * -t2 + 1.0 / 40320.0;                       // 1/8!
    pc = pc * -t2 + 1.0 / 720.0;                         // 1/6!
    pc = pc * -t2 + 1.0 / 24.0;                          // 1/4!
    pc = pc * -t2 + 0.5;                                 // 1/2!
    omc = t2 * pc;
}

// 1/sqrt(x) for x > 0 in FP64: hardware estimate refined by two Newton steps
__device__ inline double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

// One colour class: every spin takes an implicit-midpoint Rodrigues rotation
// over tau = dt/2 in the field of its (other-colour) neighbours, its own
// anisotropy/onsite terms at the midpoint, the Zeeman field and the noise.
// Eight lanes share a spin: they split the neighbour gather (couplings stored
// in colour-list order, so a wavefront reads contiguous records), reduce, and
// then run the midpoint iteration in lockstep; lane 0 stores the result.
// Latency is what bounds a colour class, so the loads are issued in two
// waves: everything indexed by the colour-list position (atom, replica,
// coupling count, self terms, the first four coupling slots of each lane,
// read whether or not they are in use and masked afterwards), then the
// neighbours' spins, the spin itself, its noise and the replica record.
constexpr int SWEEP_R0 = 4;    // coupling slots per lane loaded up front (32 per spin)

// turns = 2 takes the colour twice in a row (the end of the ascending and the
// start of the descending pass): the neighbour field is the same for both
// rotations, the second starts from the first one's result.
template <typename real>
__global__ void __launch_bounds__(256) k_sweep(Sys S, Work<real> W, int base, int count, int turns) {
    const int lane = threadIdx.x & 7;
    const int t = blockIdx.x * 32 + (threadIdx.x >> 3);
    if (t >= count) return;
    const int p = base + t;
    const size_t lf = S.N_fe;
    // first wave of loads
    const int i = S.col_idx[p];
    const int r = S.col_rid[p];
    const int nc = W.cpl_n[p];
    const real *o = W.selfc + (size_t)p * 8;
    const double Axx = o[0], Ayy = o[1], Azz = o[2], Axy = o[3], Axz = o[4], Ayz = o[5], os = o[6];
    int cj[SWEEP_R0];
    double cv[SWEEP_R0][6];
#pragma unroll
    for (int k = 0; k < SWEEP_R0; k++) {
        const size_t q = (size_t)(lane + 8 * k) * lf + p;
        cj[k] = W.cpl_j[q];
        const real *c = W.cpl + q * 6;
#pragma unroll
        for (int x = 0; x < 6; x++) cv[k][x] = c[x];
    }
    // second wave
    const RepDev &R = S.rep[r];
    const d4 e = S.eta[i];
    const d4 s4 = S.spin[i];
    double hx = 0, hy = 0, hz = 0;
    d4 sj[SWEEP_R0];
#pragma unroll
    for (int k = 0; k < SWEEP_R0; k++) sj[k] = S.spin[lane + 8 * k < nc ? cj[k] : i];
#pragma unroll
    for (int k = 0; k < SWEEP_R0; k++) {
        if (lane + 8 * k >= nc) continue;
        const double J = cv[k][0], D = cv[k][1], K = cv[k][2], rx = cv[k][3], ry = cv[k][4], rz = cv[k][5];
        const double sr = sj[k].x * rx + sj[k].y * ry + sj[k].z * rz;
        hx -= J * sj[k].x + D * (sj[k].y * rz - sj[k].z * ry) + K * sr * rx;
        hy -= J * sj[k].y + D * (sj[k].z * rx - sj[k].x * rz) + K * sr * ry;
        hz -= J * sj[k].z + D * (sj[k].x * ry - sj[k].y * rx) + K * sr * rz;
    }
    // spins with more than 8 * SWEEP_R0 couplings
    for (int s = lane + 8 * SWEEP_R0; s < nc; s += 8) {
        const int j = W.cpl_j[(size_t)s * lf + p];
        const real *c = W.cpl + ((size_t)s * lf + p) * 6;
        const double J = c[0], D = c[1], K = c[2], rx = c[3], ry = c[4], rz = c[5];
        const d4 v = S.spin[j];
        const double sr = v.x * rx + v.y * ry + v.z * rz;
        hx -= J * v.x + D * (v.y * rz - v.z * ry) + K * sr * rx;
        hy -= J * v.y + D * (v.z * rx - v.x * rz) + K * sr * ry;
        hz -= J * v.z + D * (v.x * ry - v.y * rx) + K * sr * rz;
    }
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        hx += __shfl_xor(hx, m);
        hy += __shfl_xor(hy, m);
        hz += __shfl_xor(hz, m);
    }
    if (!R.active) return;
    const double fr = ramp_frac(R), zs = R.mu_s * MUB;
    hx += zs * (R.B0[0] + (R.B1[0] - R.B0[0]) * fr) + e.x;
    hy += zs * (R.B0[1] + (R.B1[1] - R.B0[1]) * fr) + e.y;
    hz += zs * (R.B0[2] + (R.B1[2] - R.B0[2]) * fr) + e.z;
    const double al = R.alpha, inv = 1.0 / (1.0 + al * al), tau = 0.5 * R.dt / HBAR;
    const double tol = R.mid_tol;
    const int cap = R.mid_cap;
    double sx = s4.x, sy = s4.y, sz = s4.z;
    double yx = sx, yy = sy, yz = sz;
    for (int turn = 0; turn < turns; turn++) {
    if (turn) {
        sx = yx;
        sy = yy;
        sz = yz;
    }
    for (int it = 0; it < cap; it++) {
        double mx = sx + yx, my = sy + yy, mz = sz + yz;
        const double mn = rsqrt_nr(mx * mx + my * my + mz * mz);
        mx *= mn;
        my *= mn;
        mz *= mn;
        const double h0 = hx - 2.0 * (Axx * mx + Axy * my + Axz * mz + os * mx);
        const double h1 = hy - 2.0 * (Axy * mx + Ayy * my + Ayz * mz + os * my);
        const double h2 = hz - 2.0 * (Axz * mx + Ayz * my + Azz * mz + os * mz);
        const double wx = (h0 + al * (my * h2 - mz * h1)) * inv;
        const double wy = (h1 + al * (mz * h0 - mx * h2)) * inv;
        const double wz = (h2 + al * (mx * h1 - my * h0)) * inv;
        const double w2 = wx * wx + wy * wy + wz * wz;
        double nx, ny, nz;
        if (w2 == 0.0) {
            nx = sx;
            ny = sy;
            nz = sz;
        } else {
            const double iw = rsqrt_nr(w2);
            const double th = w2 * iw * tau;
            double sn, cs, omc;
            if (th < 1e-8) {
                sn = th - th * th * th / 6.0;
                omc = th * th / 2.0;
                cs = 1.0 - omc;
            } else if (th <= 1.0) {
                sin_omc_taylor(th, sn, omc);
                cs = 1.0 - omc;
            } else {
                sincos(th, &sn, &cs);
                omc = 1.0 - cs;
            }
            const double ux = wx * iw, uy = wy * iw, uz = wz * iw;
            const double us = ux * sx + uy * sy + uz * sz;
            nx = sx * cs + (uy * sz - uz * sy) * sn + ux * us * omc;
            ny = sy * cs + (uz * sx - ux * sz) * sn + uy * us * omc;
            nz = sz * cs + (ux * sy - uy * sx) * sn + uz * us * omc;
        }
        const double diff = fmax(fabs(nx - yx), fmax(fabs(ny - yy), fabs(nz - yz)));
        yx = nx;
        yy = ny;
        yz = nz;
        if (diff <= tol) break;
    }
    }
    if (lane == 0) {
        d4 out = {yx, yy, yz, 0.0};
        S.spin[i] = out;
    }
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
    // a replica waiting for a new colouring stops after this (exact) step
    if (R.step >= R.step_end || (R.failed & 4)) R.active = 0;
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
        const double m = mass_of(fe ? 0 : 1);
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
        }
        const double chk = p.x + p.y + p.z + vel.x + vel.y + vel.z + s.x + s.y + s.z + F.x + F.y + F.z + v[0];
        v[8] = isfinite(chk) ? 0.0 : 1.0;
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
    // slot NOBS-1 counts non-finite atoms
    if (t < NOBS) out[(size_t)r * NOBS + t] = red[t][0];
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
            if (n > 0) hipLaunchKernelGGL(k_sweep<real>, dim3(nblk(n, 32)), dim3(256), 0, st, S, W, b, n, turns);
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
