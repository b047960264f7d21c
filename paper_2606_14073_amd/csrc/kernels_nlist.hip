// kernels_nlist.hip -- Verlet cell/neighbour lists on the device.
//
// Atoms are binned into cells at least r_list = rc + skin wide; every atom
// scans its (up to) 27 surrounding cells, keeps candidates within r_list by
// minimum image and stores a full list (both i->j and j->i) sorted by atom
// index, so the order of every later neighbour sum is fixed and independent
// of thread timing. Lists are rebuilt only when some atom moved more than
// skin/2 since the last build (the rebuild flag is raised on the device and
// every rebuild kernel exits at once when it is clear).
#include "engine.h"

namespace nep {

namespace {

constexpr int BLK = 64;

__device__ inline int cell_coord(double x, const RepDev &R, int a) {
    double u = x - R.cell_lo[a];
    if (R.pbc[a]) u -= R.box[a] * floor(u / R.box[a]);
    int c = (int)floor(u / R.cell_w[a]);
    if (c < 0) c = 0;
    if (c >= R.nc[a]) c = R.nc[a] - 1;
    return c;
}

__global__ void k_skin(Sys S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const RepDev &R = S.rep[S.rid[i]];
    double dx, dy, dz;
    min_image(R, S.pos_ref[i], S.pos[i], dx, dy, dz);
    const double h = 0.5 * R.skin;
    if (dx * dx + dy * dy + dz * dz > h * h) atomicOr(&S.flags[F_REBUILD], 1);
}

__global__ void k_cells_zero(Sys S) {
    if (S.flags[F_REBUILD] == 0) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < S.n_cells; c += gridDim.x * blockDim.x) {
        S.cell_cnt[c] = 0;
        S.cell_fill[c] = 0;
    }
}

__global__ void k_cells_count(Sys S) {
    if (S.flags[F_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const RepDev &R = S.rep[S.rid[i]];
    const d4 p = S.pos[i];
    const int c = R.cell_base + (cell_coord(p.x, R, 0) * R.nc[1] + cell_coord(p.y, R, 1)) * R.nc[2] +
                  cell_coord(p.z, R, 2);
    S.cell_of[i] = c;
    atomicAdd(&S.cell_cnt[c], 1);
}

// exclusive scan of the cell counts by one workgroup of 1024 threads
__global__ void __launch_bounds__(1024) k_cells_scan(Sys S) {
    if (S.flags[F_REBUILD] == 0) return;
    __shared__ int part[1024];
    const int t = threadIdx.x, n = S.n_cells;
    const int per = (n + 1023) / 1024;
    const int b = t * per, e = min(n, b + per);
    int s = 0;
    for (int c = b; c < e; c++) s += S.cell_cnt[c];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t ? part[t - 1] : 0;
    for (int c = b; c < e; c++) {
        S.cell_start[c] = run;
        run += S.cell_cnt[c];
    }
}

__global__ void k_cells_fill(Sys S) {
    if (S.flags[F_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const int c = S.cell_of[i];
    const int k = atomicAdd(&S.cell_fill[c], 1);
    S.cell_atoms[S.cell_start[c] + k] = i;
}

__device__ inline void axis_offsets(const RepDev &R, int a, int c, int off[3], int &n) {
    n = 0;
    if (R.pbc[a]) {
        const int m = R.nc[a];
        if (m >= 3) {
            off[n++] = (c + m - 1) % m;
            off[n++] = c;
            off[n++] = (c + 1) % m;
        } else if (m == 2) {
            off[n++] = c;
            off[n++] = 1 - c;
        } else {
            off[n++] = c;
        }
    } else {
        for (int d = -1; d <= 1; d++)
            if (c + d >= 0 && c + d < R.nc[a]) off[n++] = c + d;
    }
}

__device__ inline void sort_row(int *row, int n) {
    // row is k-major in LDS: element k at row[k * BLK]
    for (int x = 1; x < n; x++) {
        int v = row[x * BLK], y = x - 1;
        while (y >= 0 && row[y * BLK] > v) {
            row[(y + 1) * BLK] = row[y * BLK];
            y--;
        }
        row[(y + 1) * BLK] = v;
    }
}

// Fallback, one lane per atom, for the atoms of cells whose 27-cell
// neighbourhood holds more candidates than the cell kernel stages: the
// radial-set list sorted by atom index in LDS; the angular-set list is the
// sorted radial row filtered by distance (rc_A + skin < rc_R + skin), so it
// comes out sorted and each of its entries knows its radial slot (a2r).
__global__ void __launch_bounds__(BLK) k_build(Sys S, double rl2R, double rl2A) {
    if (S.flags[F_REBUILD] == 0) return;
    __shared__ int rowR[MAXR * BLK];
    const int t = threadIdx.x;
    const int i = blockIdx.x * BLK + t;
    if (i >= S.N) return;
    if (S.cell_fill[S.cell_of[i]] == 0) return;   // built by the cell kernel
    const RepDev &R = S.rep[S.rid[i]];
    const Img g = img_of(R);
    const d4 pi = S.pos[i];
    int cx = cell_coord(pi.x, R, 0), cy = cell_coord(pi.y, R, 1), cz = cell_coord(pi.z, R, 2);
    int ox[3], oy[3], oz[3], nx, ny, nz;
    axis_offsets(R, 0, cx, ox, nx);
    axis_offsets(R, 1, cy, oy, ny);
    axis_offsets(R, 2, cz, oz, nz);
    int nr = 0;
    for (int a = 0; a < nx; a++)
        for (int b = 0; b < ny; b++)
            for (int c = 0; c < nz; c++) {
                const int cell = R.cell_base + (ox[a] * R.nc[1] + oy[b]) * R.nc[2] + oz[c];
                const int beg = S.cell_start[cell], cnt = S.cell_cnt[cell];
                // the next atom's index and position are loaded one ahead
                int jn = cnt > 0 ? S.cell_atoms[beg] : 0;
                d4 pn = S.pos[jn];
                for (int q = 0; q < cnt; q++) {
                    const int j = jn;
                    const d4 pj = pn;
                    if (q + 1 < cnt) {
                        jn = S.cell_atoms[beg + q + 1];
                        pn = S.pos[jn];
                    }
                    if (j == i) continue;
                    double dx, dy, dz;
                    min_image(g, pi, pj, dx, dy, dz);
                    if (dx * dx + dy * dy + dz * dz < rl2R) {
                        if (nr < MAXR) rowR[nr * BLK + t] = j;
                        nr++;
                    }
                }
            }
    bool over = nr > MAXR;
    nr = min(nr, MAXR);
    sort_row(rowR + t, nr);
    int fe = 0, na = 0, fea = 0;
    for (int s = 0; s < nr; s++) {
        const int j = rowR[s * BLK + t];
        S.nbrR[(size_t)s * S.N + i] = j;
        fe += j < S.N_fe;
        double dx, dy, dz;
        min_image(g, pi, S.pos[j], dx, dy, dz);
        if (dx * dx + dy * dy + dz * dz < rl2A) {
            if (na < MAXA) {
                S.nbrA[(size_t)na * S.N + i] = j;
                S.a2r[(size_t)na * S.N + i] = s;
            }
            na++;
            fea += j < S.N_fe;
        }
    }
    over |= na > MAXA;
    na = min(na, MAXA);
    fea = min(fea, na);
    S.cntR[i] = nr;
    S.cntFeR[i] = fe;
    S.cntA[i] = na;
    S.cntFeA[i] = fea;
    if (over || (S.mag && i < S.N_fe && fe > MAXFE)) {
        atomicOr(&S.flags[F_OVERFLOW], 1);
        atomicOr(&S.rep[S.rid[i]].failed, 1);
    }
    S.pos_ref[i] = pi;
}

// One workgroup per cell: the candidates of its 27-cell neighbourhood are
// staged in LDS, sorted by atom index (bitonic), and their positions loaded
// once; then 8 lanes per home atom split the sorted candidates into
// contiguous eighths, count their hits, take offsets by a prefix over the
// eight lanes and write them in order: every radial row comes out sorted,
// the angular row is its sub-row within rc_A + skin, with its radial slots.
// Lists are the same as the per-atom kernel's. A neighbourhood with more than
// CAND candidates is left to that kernel (cell_fill[cell] = 1).
constexpr int CAND = 1024;
constexpr int BC = 256, LPA = 8;

__global__ void __launch_bounds__(BC) k_build_cells(Sys S, double rl2R, double rl2A) {
    if (S.flags[F_REBUILD] == 0) return;
    __shared__ int cidx[CAND];
    __shared__ double cpx[CAND], cpy[CAND], cpz[CAND];
    __shared__ int s_cell[27], s_beg[28], s_nc;
    const int home = blockIdx.x, tid = threadIdx.x;
    const int hbeg = S.cell_start[home], hcnt = S.cell_cnt[home];
    if (hcnt == 0) {
        if (tid == 0) S.cell_fill[home] = 0;
        return;
    }
    const RepDev &R = S.rep[S.rid[S.cell_atoms[hbeg]]];
    if (tid == 0) {
        const int lc = home - R.cell_base;
        const int cx = lc / (R.nc[1] * R.nc[2]), cy = (lc / R.nc[2]) % R.nc[1], cz = lc % R.nc[2];
        int ox[3], oy[3], oz[3], nx, ny, nz;
        axis_offsets(R, 0, cx, ox, nx);
        axis_offsets(R, 1, cy, oy, ny);
        axis_offsets(R, 2, cz, oz, nz);
        int k = 0, tot = 0;
        for (int a = 0; a < nx; a++)
            for (int b = 0; b < ny; b++)
                for (int c = 0; c < nz; c++) {
                    const int cell = R.cell_base + (ox[a] * R.nc[1] + oy[b]) * R.nc[2] + oz[c];
                    s_cell[k] = cell;
                    s_beg[k] = tot;
                    tot += S.cell_cnt[cell];
                    k++;
                }
        s_beg[k] = tot;
        s_nc = k;
    }
    __syncthreads();
    const int nc = s_nc, n = s_beg[nc];
    if (n > CAND) {
        if (tid == 0) S.cell_fill[home] = 1;
        return;
    }
    int P = 1;
    while (P < n) P <<= 1;
    for (int k = tid; k < P; k += BC) {
        int v = 0x7fffffff;   // padding sorts last
        if (k < n) {
            int q = 0;
            while (s_beg[q + 1] <= k) q++;
            v = S.cell_atoms[S.cell_start[s_cell[q]] + (k - s_beg[q])];
        }
        cidx[k] = v;
    }
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int t = tid; t < P; t += BC) {
                const int u = t ^ j;
                if (u > t) {
                    const int a = cidx[t], b = cidx[u];
                    if ((a > b) == ((t & kk) == 0)) {
                        cidx[t] = b;
                        cidx[u] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int k = tid; k < n; k += BC) {
        const d4 p = S.pos[cidx[k]];
        cpx[k] = p.x;
        cpy[k] = p.y;
        cpz[k] = p.z;
    }
    __syncthreads();
    const Img g = img_of(R);   // the box in registers for the candidate loops
    const int lane = tid % LPA;
    const int lo = lane * n / LPA, hi = (lane + 1) * n / LPA;
    for (int h0 = 0; h0 < hcnt; h0 += BC / LPA) {
        const int h = h0 + tid / LPA;
        const bool act = h < hcnt;
        const int i = act ? S.cell_atoms[hbeg + h] : 0;
        const d4 pi = S.pos[i];
        // pass 1: hits of this lane's eighth
        int cR = 0, cRf = 0, cA = 0, cAf = 0;
        for (int k = lo; k < hi && act; k++) {
            const int j = cidx[k];
            if (j == i) continue;
            double dx, dy, dz;
            min_image(g, pi, d4{cpx[k], cpy[k], cpz[k], 0.0}, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rl2R) {
                cR++;
                cRf += j < S.N_fe;
                if (r2 < rl2A) {
                    cA++;
                    cAf += j < S.N_fe;
                }
            }
        }
        // exclusive offsets over the atom's eight lanes
        int oR = cR, oA = cA;
#pragma unroll
        for (int d = 1; d < LPA; d <<= 1) {
            const int uR = __shfl_up(oR, d, LPA), uA = __shfl_up(oA, d, LPA);
            if (lane >= d) {
                oR += uR;
                oA += uA;
            }
        }
        int fR = cRf, fA = cAf;
#pragma unroll
        for (int d = 1; d < LPA; d <<= 1) {
            fR += __shfl_xor(fR, d, LPA);
            fA += __shfl_xor(fA, d, LPA);
        }
        const int nr = __shfl(oR, LPA - 1, LPA), na = __shfl(oA, LPA - 1, LPA);
        oR -= cR;
        oA -= cA;
        // pass 2: write the hits in order
        for (int k = lo; k < hi && act; k++) {
            const int j = cidx[k];
            if (j == i) continue;
            double dx, dy, dz;
            min_image(g, pi, d4{cpx[k], cpy[k], cpz[k], 0.0}, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rl2R) {
                if (oR < MAXR) S.nbrR[(size_t)oR * S.N + i] = j;
                if (r2 < rl2A) {
                    if (oA < MAXA) {
                        S.nbrA[(size_t)oA * S.N + i] = j;
                        S.a2r[(size_t)oA * S.N + i] = oR;
                    }
                    oA++;
                }
                oR++;
            }
        }
        if (act && lane == 0) {
            const bool over = nr > MAXR || na > MAXA;
            S.cntR[i] = min(nr, MAXR);
            S.cntFeR[i] = min(fR, MAXR);
            S.cntA[i] = min(na, MAXA);
            S.cntFeA[i] = min(fA, MAXA);
            if (over || (S.mag && i < S.N_fe && fR > MAXFE)) {
                atomicOr(&S.flags[F_OVERFLOW], 1);
                atomicOr(&S.rep[S.rid[i]].failed, 1);
            }
            S.pos_ref[i] = pi;
        }
    }
    if (tid == 0) S.cell_fill[home] = 0;
}

__device__ inline int find_sorted(const int *nbr, int N, int row, int n, int key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int v = nbr[(size_t)mid * N + row];
        if (v < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && nbr[(size_t)lo * N + row] == key) ? lo : -1;
}

// reverse slots (where i sits in j's list), angular->radial slot map, and the
// colouring check. A same-colour spin pair inside rc_R would be updated
// concurrently by the sweep although coupled: the replica fails (bit 2). A
// same-colour pair in the list shell (rc_R, rc_R + skin] is not coupled yet
// and cannot come inside rc_R before the next rebuild, so the step stays
// exact; the replica is paused at the end of the step for recolouring (bit 4).
__global__ void k_rev(Sys S) {
    if (S.flags[F_REBUILD] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const int na = S.cntA[i];
    int bad = 0;
    // reverse radial slots: used by the spin couplings only (spin-carrying pairs)
    const int nm = S.mag && i < S.N_fe ? min(S.cntFeR[i], MAXFE) : 0;
    for (int s = 0; s < nm; s++) {
        const int j = S.nbrR[(size_t)s * S.N + i];
        const int r = find_sorted(S.nbrR, S.N, j, S.cntR[j], i);
        bad |= r < 0;
        S.revR[(size_t)s * S.N + i] = r < 0 ? 0 : r;
    }
    for (int s = 0; s < na; s++) {
        const int j = S.nbrA[(size_t)s * S.N + i];
        const int r = find_sorted(S.nbrA, S.N, j, S.cntA[j], i);
        bad |= r < 0;
        S.revA[(size_t)s * S.N + i] = r < 0 ? 0 : r;
    }
    if (bad) {
        atomicOr(&S.flags[F_OVERFLOW], 2);
        atomicOr(&S.rep[S.rid[i]].failed, 1);
    }
    if (S.colour && i < S.N_fe && S.colour[i] >= 0) {
        const int ci = S.colour[i];
        const int nfe = S.cntFeR[i];
        const RepDev &R = S.rep[S.rid[i]];
        const d4 pi = S.pos[i];
        int conflict = 0;
        for (int s = 0; s < nfe; s++) {
            const int j = S.nbrR[(size_t)s * S.N + i];
            if (S.colour[j] == ci) {
                double dx, dy, dz;
                min_image(R, pi, S.pos[j], dx, dy, dz);
                conflict |= dx * dx + dy * dy + dz * dz < RC_R * RC_R ? 2 : 4;
            }
        }
        if (conflict) {
            atomicOr(&S.flags[F_COLOUR], 1);
            atomicOr(&S.rep[S.rid[i]].failed, conflict);
        }
    }
}

__global__ void k_rebuild_done(Sys S) {
    if (threadIdx.x == 0 && blockIdx.x == 0) S.flags[F_REBUILD] = 0;
}

inline int nblk(int n, int b) { return (n + b - 1) / b; }

}  // namespace

void launch_skin_check(const Sys &S, hipStream_t st) {
    if (S.N == 0) return;
    hipLaunchKernelGGL(k_skin, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
}

void launch_rebuild(const Sys &S, double r_listR, double r_listA, hipStream_t st) {
    if (S.N == 0) return;
    hipLaunchKernelGGL(k_cells_zero, dim3(std::min(nblk(S.n_cells, 256), 1024)), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_cells_count, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_cells_scan, dim3(1), dim3(1024), 0, st, S);
    hipLaunchKernelGGL(k_cells_fill, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_build_cells, dim3(S.n_cells), dim3(BC), 0, st, S, r_listR * r_listR, r_listA * r_listA);
    hipLaunchKernelGGL(k_build, dim3(nblk(S.N, BLK)), dim3(BLK), 0, st, S, r_listR * r_listR,
                       r_listA * r_listA);
    hipLaunchKernelGGL(k_rev, dim3(nblk(S.N, 256)), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_rebuild_done, dim3(1), dim3(64), 0, st, S);
}

}  // namespace nep
