// engine.cpp -- host runtime of the spin-lattice NEP library: model upload,
// the batch engine (replica layout in HBM, step sequencing on one HIP stream)
// and the C ABI declared in nepspin.h, including the replica server.
#include "engine.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "nepspin.h"
#include "scratch.h"

using namespace nep;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

extern "C" const char *sl_last_error(void) { return g_err.c_str(); }

#define HIPCHK(x)                                                                                \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess) return fail(SL_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static int dalloc(T **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SL_E_OOM, std::string("hipMalloc of ") + std::to_string(n * sizeof(T)) + " bytes failed");
    }
    return SL_OK;
}

template <typename T>
static void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// model
// ---------------------------------------------------------------------------

struct nep_model {
    std::vector<double> p;          // spin-aware layout (a structural-only model is expanded)
    bool structural = false;
    double zbl[4] = {0, 0, 0, 0};   // short-range term: Z_0, Z_1, r_inner, r_outer (r_outer 0: off)
    double landau[2] = {0, 0};      // onsite moment-length term a|s|^2 + b|s|^4 of spin carriers
    double *d64 = nullptr;
    float *d32 = nullptr;
    ModelDev<double> m64{};
    ModelDev<float> m32{};
    std::mutex eval_mu;
    struct Engine *eval_eng[2] = {nullptr, nullptr};
};

// e^2/(4 pi eps0) in eV A, the Bohr radius in A (CODATA), and the universal
// screening length a = 0.8854 a_Bohr / (Z_i^0.23 + Z_j^0.23) of Ziegler,
// Biersack and Littmark
constexpr double K_COULOMB = 14.399645;
constexpr double A_BOHR = 0.529177210903;

template <typename real>
static void model_layout(const std::vector<double> &p, const double *zbl, std::vector<real> &h) {
    h.assign(MODEL_DEV, real(0));
    size_t o = 0;
    auto copy = [&](int off, int n) {
        for (int k = 0; k < n; k++) h[o + k] = (real)p[off + k];
        o += n;
    };
    copy(P_CR, 324);
    copy(P_CA, 252);
    copy(P_CEX, 324);
    copy(P_CDM, 324);
    copy(P_CAN, 324);
    copy(P_CSI, 324);
    copy(P_CSA, 252);
    for (int t = 0; t < 2; t++) {
        const double *W0 = p.data() + P_MLP + t * P_MLP_STRIDE;
        for (int d = 0; d < ND; d++)
            for (int hh = 0; hh < NH; hh++) h[o + (size_t)d * NH + hh] = (real)W0[hh * ND + d];
        o += (size_t)DP * NH;
    }
    for (int t = 0; t < 2; t++)
        for (int hh = 0; hh < NH; hh++) h[o++] = (real)p[P_MLP + t * P_MLP_STRIDE + NH * ND + hh];
    for (int t = 0; t < 2; t++)
        for (int hh = 0; hh < NH; hh++) h[o++] = (real)p[P_MLP + t * P_MLP_STRIDE + NH * ND + NH + hh];
    for (int t = 0; t < 2; t++) h[o++] = (real)p[P_MLP + t * P_MLP_STRIDE + NH * ND + 2 * NH];
    if (zbl[3] > 0) {
        for (int tau = 0; tau < 4; tau++) {
            const double zi = zbl[tau >> 1], zj = zbl[tau & 1];
            h[M_ZBL + tau] = (real)(K_COULOMB * zi * zj);
            h[M_ZBL + 4 + tau] = (real)((std::pow(zi, 0.23) + std::pow(zj, 0.23)) / (0.8854 * A_BOHR));
        }
        h[M_ZBL + 8] = (real)zbl[2];
        h[M_ZBL + 9] = (real)zbl[3];
        h[M_ZBL + 10] = (real)(M_PI / (zbl[3] - zbl[2]));
        h[M_ZBL + 11] = real(1);
    }
}

template <typename real>
static ModelDev<real> model_ptrs(real *base) {
    ModelDev<real> m;
    size_t o = 0;
    m.cR = base + o; o += 324;
    m.cA = base + o; o += 252;
    m.cEX = base + o; o += 324;
    m.cDM = base + o; o += 324;
    m.cAN = base + o; o += 324;
    m.cSI = base + o; o += 324;
    m.cSA = base + o; o += 252;
    m.W0 = base + o; o += 2 * (size_t)DP * NH;
    m.b0 = base + o; o += 2 * NH;
    m.w1 = base + o; o += 2 * NH;
    m.b1 = base + o; o += 2;
    return m;
}

// ---------------------------------------------------------------------------
// replica and engine
// ---------------------------------------------------------------------------

struct Replica {
    uint64_t id = 0;
    int64_t n = 0, n_fe = 0;
    std::vector<int> fe_idx, ge_idx;       // caller index of internal atoms
    std::vector<int> colour_fe;            // colour of each spin carrier (internal order)
    int ncol = 0;
    RepDev dev{};                          // parameters (host copy)
    int fe_off = -1, ge_off = -1;          // position in the current layout, -1 when not resident
    int slot = -1;                         // replica index in the layout
    std::vector<double> pos, vel, spin;    // caller order, used before admission / after eviction
    int64_t n_steps = 0, steps_done = 0, step0 = 0;
    int state = SL_QUEUED, error = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<double> lat;
    double obs_last[NOBS] = {0};
    int64_t obs_step = 0;
    size_t bytes = 0;
    int64_t n_recolour = 0;                // colourings replaced since creation
    int last_passes = 0;                   // self-consistent: sweep passes of the last step run
    double last_change = 0;                // and the change of its last pass
    bool need_recolour = false;            // paused on a colour conflict in the list shell
};

static size_t bytes_per_atom(sl_precision prec) {
    const size_t rs = prec == SL_FP64 ? 8 : 4;
    size_t b = 9 * sizeof(d4) + 9 * 4 + 2 * MAXR * 4 + 3 * MAXA * 4;
    b += rs * (2 * DP + 1 + NA * NAB + 12 + RCOEF + 4 * MAXA);
    b += (rs * (MAXFE * 7 + MCOEF + 14) + 4 * (MAXFE + 3) + sizeof(d4)) / 2 + 64;   // per spin carrier, half the atoms
    return b;
}

extern "C" size_t sl_replica_bytes(int64_t n_atoms, sl_precision prec) {
    if (n_atoms < 0) return 0;
    return bytes_per_atom(prec) * (size_t)n_atoms + 4096;
}

struct Engine {
    // Device arrays come from hipMalloc, or, when `arena` is set, are carved
    // in order from that caller-provided region (never freed here; the stream
    // is then the caller's, no stream or event is created).
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    template <typename T>
    int get(T **p, size_t n) {
        if (!arena) return dalloc(p, n);
        if (n == 0) n = 1;
        const size_t bytes = (n * sizeof(T) + 255) & ~(size_t)255;
        if (arena_used + bytes > arena_cap) {
            *p = nullptr;
            return fail(SL_E_OOM, "system too large for the static scratch area (" + std::to_string(arena_cap >> 20) +
                                      " MiB per GPU): use nep_spin_eval");
        }
        *p = reinterpret_cast<T *>(arena + arena_used);
        arena_used += bytes;
        return SL_OK;
    }
    template <typename T>
    void put(T *&p) {
        if (!arena) dfree(p);
        p = nullptr;
    }

    nep_model *M = nullptr;
    sl_precision prec = SL_FP64;
    int K_corr = 1;
    double sc_tol = 0;     // > 0: corrector passes repeated until the spins settle (single replica)
    int sc_max = 0;
    int sc_depth = 0;      // > 0: Anderson mixing over that many residual differences
    double sc_reg = 0;
    std::vector<int> log_passes;       // self-consistent: per step since the last clear, sweep passes
    std::vector<double> log_change;    // and the residual of the last pass
    hipStream_t st = nullptr;
    bool own_stream = false;

    std::vector<Replica *> reps;
    int N = 0, N_fe = 0, n_cells = 0;
    size_t cap = 0, cap_fe = 0, cap_cells = 0, cap_rep = 0, cap_chunks = 0;

    // device arrays
    int *rid = nullptr, *orig = nullptr, *colour = nullptr;
    RepDev *rep = nullptr;
    d4 *pos = nullptr, *vel = nullptr, *spin = nullptr, *force = nullptr, *field = nullptr, *pos_ref = nullptr,
       *spin_n = nullptr, *spin_hat = nullptr, *eta = nullptr;
    d4 *sc_x = nullptr, *sc_f = nullptr, *sc_g = nullptr, *sc_dF = nullptr, *sc_dG = nullptr;
    double *sc_part = nullptr, *sc_out = nullptr;
    int *nbrR = nullptr, *cntR = nullptr, *cntFeR = nullptr, *revR = nullptr;
    int *nbrA = nullptr, *cntA = nullptr, *cntFeA = nullptr, *revA = nullptr, *a2r = nullptr;
    int *cell_of = nullptr, *cell_cnt = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *cell_atoms = nullptr;
    int *flags = nullptr;
    int *act_buf = nullptr;    // [2 cap_rep] 'active' words to set on a re-layout (-1: leave)
    d4 *stage_buf = nullptr;   // staging of resident state across a re-layout (grow-only)
    size_t stage_cap = 0;
    int *src_buf = nullptr;    // re-layout: old row of each new row (grow-only)
    size_t src_cap = 0;
    void *work = nullptr;      // real-typed work arrays, one allocation
    size_t work_bytes = 0;
    Work<double> w64{};
    Work<float> w32{};
    Chunk *chunks = nullptr;
    int *chunk_ptr = nullptr, *col_idx = nullptr, *colpos = nullptr, *col_rid = nullptr, *cpl_j = nullptr,
        *cpl_n = nullptr;
    double *partial = nullptr, *obs = nullptr;
    size_t cap_obs = 0, cap_col = 0;
    int n_chunks = 0;
    std::vector<int> col_ptr;

    // kernel-group timing (sl_profile_enable)
    unsigned prof_mask = 0;
    std::vector<hipEvent_t> prof_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_open;
    size_t prof_used = 0;
    double prof_ms[SL_NPROF] = {0};
    int64_t prof_n[SL_NPROF] = {0};

    hipEvent_t prof_event() {
        if (prof_used == prof_pool.size()) {
            hipEvent_t e;
            (void)hipEventCreate(&e);
            prof_pool.push_back(e);
        }
        return prof_pool[prof_used++];
    }
    struct ProfScope {
        Engine *e;
        int g;
        hipEvent_t a{}, b{};
        ProfScope(Engine *e_, int g_) : e(e_), g(g_) {
            if (e->prof_mask & (1u << g)) {
                a = e->prof_event();
                b = e->prof_event();
                (void)hipEventRecord(a, e->st);
            }
        }
        ~ProfScope() {
            if (e->prof_mask & (1u << g)) {
                (void)hipEventRecord(b, e->st);
                e->prof_open.push_back({g, {a, b}});
            }
        }
    };
    // after a stream synchronisation: fold the recorded pairs into the totals
    void prof_collect() {
        for (auto &x : prof_open) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, x.second.first, x.second.second) == hipSuccess) {
                prof_ms[x.first] += ms;
                prof_n[x.first] += 1;
            }
        }
        prof_open.clear();
        prof_used = 0;
    }

    ~Engine() { release(); }

    void release() {
        put(rid); put(orig); put(colour); put(rep);
        put(pos); put(vel); put(spin); put(force); put(field); put(pos_ref);
        put(spin_n); put(spin_hat); put(eta);
        put(sc_x); put(sc_f); put(sc_g); put(sc_dF); put(sc_dG); put(sc_part); put(sc_out);
        put(nbrR); put(cntR); put(cntFeR); put(revR);
        put(nbrA); put(cntA); put(cntFeA); put(revA); put(a2r);
        put(cell_of); put(cell_cnt); put(cell_start); put(cell_fill); put(cell_atoms);
        put(flags); put(chunks); put(chunk_ptr); put(col_idx); put(colpos); put(col_rid); put(cpl_j); put(cpl_n);
        put(partial); put(obs); put(act_buf);
        if (work && !arena) (void)hipFree(work);
        work = nullptr;
        if (stage_buf) (void)hipFree(stage_buf);
        stage_buf = nullptr;
        stage_cap = 0;
        if (src_buf) (void)hipFree(src_buf);
        src_buf = nullptr;
        src_cap = 0;
        cap = cap_fe = cap_cells = cap_rep = cap_chunks = cap_obs = cap_col = 0;
        for (auto e : prof_pool) (void)hipEventDestroy(e);
        prof_pool.clear();
        if (own_stream && st) (void)hipStreamDestroy(st);
        st = nullptr;
        own_stream = false;
    }

    Sys sys() const {
        Sys S;
        S.N = N;
        S.N_fe = N_fe;
        S.mag = M && M->structural ? 0 : 1;
        S.n_rep = (int)reps.size();
        S.n_cells = n_cells;
        S.rid = rid;
        S.orig = orig;
        S.rep = rep;
        S.pos = pos; S.vel = vel; S.spin = spin; S.force = force; S.field = field; S.pos_ref = pos_ref;
        S.spin_n = spin_n; S.spin_hat = spin_hat; S.eta = eta;
        S.sc_x = sc_x; S.sc_f = sc_f; S.sc_g = sc_g; S.sc_dF = sc_dF; S.sc_dG = sc_dG;
        S.sc_part = sc_part; S.sc_out = sc_out;
        S.colour = colour;
        S.col_idx = col_idx;
        S.colpos = colpos;
        S.col_rid = col_rid;
        S.nbrR = nbrR; S.cntR = cntR; S.cntFeR = cntFeR; S.revR = revR;
        S.nbrA = nbrA; S.cntA = cntA; S.cntFeA = cntFeA; S.revA = revA; S.a2r = a2r;
        S.cell_of = cell_of; S.cell_cnt = cell_cnt; S.cell_start = cell_start; S.cell_fill = cell_fill;
        S.cell_atoms = cell_atoms;
        S.flags = flags;
        return S;
    }

    int ensure_stream() {
        if (!st && !arena) {
            HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            own_stream = true;
        }
        return SL_OK;
    }

    template <typename real>
    void carve(Work<real> &w, size_t c, size_t cf) {
        real *b = (real *)work;
        size_t o = 0;
        auto take = [&](size_t n) {
            real *p = b + o;
            o += (n + 63) & ~(size_t)63;
            return p;
        };
        w.q = take(c * DP);
        w.Fp = take(c * DP);
        w.Ei = take(c);
        w.AB = take(c * NA * NAB);
        w.rcoef = take(c * RCOEF);
        w.mcoef = take(cf * MCOEF);
        w.ownM = take(cf * 6);
        w.pbA = take((size_t)MAXA * c * 4);
        w.ownR = take(c * 6);
        w.ownA = take(c * 6);
        w.csa = take((size_t)MAXFE * cf);
        w.cpl = take((size_t)MAXFE * cf * 6);
        w.selfc = take(cf * 8);
        w.cpl_j = cpl_j;
        w.cpl_n = cpl_n;
    }

    static size_t work_count(size_t c, size_t cf) {
        auto r = [](size_t n) { return (n + 63) & ~(size_t)63; };
        return r(c * DP) * 2 + r(c) + r(c * NA * NAB) + r(c * RCOEF) + r(cf * MCOEF) +
               r(cf * 6) + r((size_t)MAXA * c * 4) + 2 * r(c * 6) + r((size_t)MAXFE * cf) + r((size_t)MAXFE * cf * 6) +
               r(cf * 8);
    }

    int reserve(size_t n, size_t nfe, size_t ncell, size_t nrep, size_t nchunk) {
        int rc;
        if (n > cap || nfe > cap_fe) {
            // headroom for later growth, except in a fixed scratch area
            size_t c = arena ? n : std::max(n, cap + cap / 4), cf = arena ? nfe : std::max(nfe, cap_fe + cap_fe / 4);
            c = std::max<size_t>(c, 64);
            cf = std::max<size_t>(cf, 64);
            put(rid); put(orig); put(colour);
            put(pos); put(vel); put(spin); put(force); put(field); put(pos_ref);
            put(spin_n); put(spin_hat); put(eta);
            put(sc_x); put(sc_f); put(sc_g); put(sc_dF); put(sc_dG); put(sc_part);
            put(nbrR); put(cntR); put(cntFeR); put(revR);
            put(nbrA); put(cntA); put(cntFeA); put(revA); put(a2r);
            put(cell_of); put(cell_atoms); put(cpl_j); put(cpl_n);
            if (work && !arena) (void)hipFree(work);
            work = nullptr;
            cap = cap_fe = 0;
            if ((rc = get(&rid, c)) || (rc = get(&orig, c)) || (rc = get(&colour, c)) ||
                (rc = get(&pos, c)) || (rc = get(&vel, c)) || (rc = get(&spin, c)) ||
                (rc = get(&force, c)) || (rc = get(&field, c)) || (rc = get(&pos_ref, c)) ||
                (rc = get(&spin_n, c)) || (rc = get(&spin_hat, c)) || (rc = get(&eta, c)) ||
                (rc = get(&nbrR, (size_t)MAXR * c)) || (rc = get(&cntR, c)) || (rc = get(&cntFeR, c)) ||
                (rc = get(&revR, (size_t)MAXR * c)) || (rc = get(&nbrA, (size_t)MAXA * c)) ||
                (rc = get(&cntA, c)) || (rc = get(&cntFeA, c)) || (rc = get(&revA, (size_t)MAXA * c)) ||
                (rc = get(&a2r, (size_t)MAXA * c)) || (rc = get(&cell_of, c)) ||
                (rc = get(&cell_atoms, c)) || (rc = get(&cpl_j, (size_t)MAXFE * cf)) ||
                (rc = get(&cpl_n, cf)) || (rc = get(&sc_x, cf)))
                return rc;
            if (sc_tol > 0 && sc_depth > 0 &&
                ((rc = get(&sc_f, cf)) || (rc = get(&sc_g, cf)) || (rc = get(&sc_dF, (size_t)sc_depth * cf)) ||
                 (rc = get(&sc_dG, (size_t)sc_depth * cf)) ||
                 (rc = get(&sc_part, (size_t)sc_part_blocks((int)cf) * SC_NK))))
                return rc;
            const size_t rs = prec == SL_FP64 ? 8 : 4;
            work_bytes = work_count(c, cf) * rs;
            if (arena) {
                char *w = nullptr;
                if ((rc = get(&w, work_bytes))) return rc;
                work = w;
                HIPCHK(hipMemsetAsync(work, 0, work_bytes, st));
            } else {
                hipError_t e = hipMalloc(&work, work_bytes);
                if (e != hipSuccess) {
                    work = nullptr;
                    (void)hipGetLastError();
                    return fail(SL_E_OOM, "hipMalloc of work arrays failed");
                }
                HIPCHK(hipMemset(work, 0, work_bytes));
            }
            cap = c;
            cap_fe = cf;
            if (prec == SL_FP64) carve(w64, c, cf);
            else carve(w32, c, cf);
        }
        if (ncell > cap_cells) {
            put(cell_cnt); put(cell_start); put(cell_fill);
            size_t c = std::max(ncell, cap_cells + cap_cells / 4);
            if ((rc = get(&cell_cnt, c)) || (rc = get(&cell_start, c)) || (rc = get(&cell_fill, c))) return rc;
            cap_cells = c;
        }
        if (nrep > cap_rep) {
            put(rep); put(chunk_ptr); put(obs); put(act_buf);
            size_t c = std::max<size_t>(nrep, 2 * cap_rep);
            if ((rc = get(&rep, c)) || (rc = get(&chunk_ptr, c + 1)) || (rc = get(&act_buf, 2 * c))) return rc;
            cap_rep = c;
            cap_obs = 0;
        }
        if (nchunk > cap_chunks) {
            put(chunks); put(partial);
            size_t c = std::max(nchunk, 2 * cap_chunks);
            if ((rc = get(&chunks, c)) || (rc = get(&partial, c * NOBS))) return rc;
            cap_chunks = c;
        }
        if (!flags) {
            if ((rc = get(&flags, NFLAGS)) || (rc = get(&sc_out, SC_OUT))) return rc;
            HIPCHK(hipMemsetAsync(flags, 0, NFLAGS * sizeof(int), st));
            HIPCHK(hipStreamSynchronize(st));
        }
        if (!col_idx || cap_col < cap_fe) {
            put(col_idx);
            put(colpos);
            put(col_rid);
            if ((rc = get(&col_idx, cap_fe)) || (rc = get(&colpos, cap_fe)) || (rc = get(&col_rid, cap_fe)))
                return rc;
            cap_col = cap_fe;
        }
        return SL_OK;
    }

    int ensure_obs(size_t nsteps) {
        size_t need = std::max<size_t>(nsteps, 1) * std::max<size_t>(reps.size(), 1) * NOBS;
        if (need > cap_obs) {
            put(obs);
            int rc = get(&obs, need);
            if (rc) return rc;
            cap_obs = need;
        }
        return SL_OK;
    }

    // cell grid of one replica (cells at least r_list wide)
    static void cell_grid(Replica &r, const double *pos_caller) {
        const double rl = RC_R + r.dev.skin;
        for (int a = 0; a < 3; a++) {
            if (r.dev.pbc[a]) {
                r.dev.nc[a] = std::max(1, (int)std::floor(r.dev.box[a] / rl));
                r.dev.cell_lo[a] = 0.0;
                r.dev.cell_w[a] = r.dev.box[a] / r.dev.nc[a];
            } else {
                double mn = 1e300, mx = -1e300;
                for (int64_t i = 0; i < r.n; i++) {
                    mn = std::min(mn, pos_caller[3 * i + a]);
                    mx = std::max(mx, pos_caller[3 * i + a]);
                }
                if (r.n == 0) mn = mx = 0;
                const double margin = 2.0 * rl;
                const double ext = (mx - mn) + 2 * margin;
                r.dev.nc[a] = std::max(1, (int)std::floor(ext / rl));
                r.dev.cell_lo[a] = mn - margin;
                r.dev.cell_w[a] = ext / r.dev.nc[a];
            }
        }
    }

    // Place replicas new_reps in a fresh layout. State of replicas already
    // resident is moved device-to-device; others are uploaded from r->pos etc.
    int set_layout(const std::vector<Replica *> &new_reps) {
        int rc;
        if ((rc = ensure_stream())) return rc;
        // old device state must survive reallocation: stage it on the host when
        // the arrays will grow, else move inside the device
        size_t n = 0, nfe = 0, ncell = 0, nchunk = 0;
        for (Replica *r : new_reps) {
            n += r->n;
            nfe += r->n_fe;
            ncell += (size_t)r->dev.nc[0] * r->dev.nc[1] * r->dev.nc[2];
            nchunk += (r->n_fe + 255) / 256 + (r->n - r->n_fe + 255) / 256;
        }
        const bool grow = n > cap || nfe > cap_fe;
        std::vector<Replica *> moved;
        for (Replica *r : reps) {
            if (std::find(new_reps.begin(), new_reps.end(), r) != new_reps.end() && r->fe_off >= 0) moved.push_back(r);
        }
        // Snapshot the resident state (the arrays may be reallocated and the
        // new ranges may overlap the old ones). On the device: the five state
        // arrays copied whole into a staging buffer and the replica records in
        // one copy, the kept replicas' rows placed afterwards by one gather
        // kernel, so that a re-layout costs a few calls however many replicas
        // stay. In host memory, replica by replica, when that buffer cannot be
        // allocated.
        const size_t n_old = moved.empty() ? 0 : (size_t)N;
        // a grow-only device buffer kept by the engine, so that admissions
        // and retirements do not allocate each time
        if (n_old && !arena && 5 * n_old > stage_cap) {
            const size_t want = 5 * std::max(n_old, stage_cap / 5 + stage_cap / 20);
            if (stage_buf) (void)hipFree(stage_buf);
            stage_buf = nullptr;
            stage_cap = 0;
            if (hipMalloc((void **)&stage_buf, want * sizeof(d4)) == hipSuccess) {
                stage_cap = want;
            } else {
                (void)hipGetLastError();
                stage_buf = nullptr;
            }
        }
        d4 *const stage = n_old && stage_buf && 5 * n_old <= stage_cap ? stage_buf : nullptr;
        std::vector<int> old_fe(moved.size()), old_ge(moved.size());
        for (size_t k = 0; k < moved.size(); k++) {
            old_fe[k] = moved[k]->fe_off;
            old_ge[k] = moved[k]->ge_off;
        }
        std::vector<std::vector<d4>> snap(stage ? 0 : moved.size() * 5);
        if (stage) {
            const d4 *src[5] = {pos, vel, spin, force, field};
            for (int a = 0; a < 5; a++)
                HIPCHK(hipMemcpyAsync(stage + a * n_old, src[a], n_old * sizeof(d4), hipMemcpyDeviceToDevice, st));
            std::vector<RepDev> old(reps.size());
            HIPCHK(hipMemcpyAsync(old.data(), rep, reps.size() * sizeof(RepDev), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (Replica *r : moved) r->dev = old[r->slot];
        }
        for (size_t k = 0; k < moved.size() && !stage; k++) {
            Replica *r = moved[k];
            d4 *src[5] = {pos, vel, spin, force, field};
            for (int a = 0; a < 5; a++) {
                snap[5 * k + a].resize(r->n);
                d4 *to = snap[5 * k + a].data();
                if (r->n_fe)
                    HIPCHK(hipMemcpyAsync(to, src[a] + r->fe_off, r->n_fe * sizeof(d4), hipMemcpyDeviceToHost, st));
                if (r->n - r->n_fe)
                    HIPCHK(hipMemcpyAsync(to + r->n_fe, src[a] + r->ge_off, (r->n - r->n_fe) * sizeof(d4),
                                          hipMemcpyDeviceToHost, st));
            }
            HIPCHK(hipMemcpyAsync(&r->dev, rep + r->slot, sizeof(RepDev), hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        (void)grow;
        for (Replica *r : reps) {
            r->fe_off = r->ge_off = -1;
            r->slot = -1;
        }
        if ((rc = reserve(n, nfe, ncell, new_reps.size(), nchunk))) return rc;
        reps = new_reps;
        N = (int)n;
        N_fe = (int)nfe;
        // offsets
        int fo = 0, go = (int)nfe, cb = 0;
        std::vector<int> h_rid(n), h_orig(n), h_col(n, -1);
        std::vector<RepDev> h_rep(reps.size());
        std::vector<Chunk> h_chunks;
        std::vector<int> h_cptr;
        int cmax = 0;
        for (size_t k = 0; k < reps.size(); k++) {
            Replica *r = reps[k];
            r->slot = (int)k;
            r->fe_off = fo;
            r->ge_off = go;
            r->dev.cell_base = cb;
            r->dev.n_atoms = (int)r->n;
            r->dev.fe_off = fo;
            r->dev.n_fe = (int)r->n_fe;
            r->dev.ge_off = go;
            r->dev.n_ge = (int)(r->n - r->n_fe);
            cb += r->dev.nc[0] * r->dev.nc[1] * r->dev.nc[2];
            h_cptr.push_back((int)h_chunks.size());
            for (int64_t a = 0; a < r->n_fe; a++) {
                h_rid[fo + a] = (int)k;
                h_orig[fo + a] = r->fe_idx[a];
                h_col[fo + a] = r->colour_fe.empty() ? -1 : r->colour_fe[a];
            }
            for (int64_t a = 0; a < r->n - r->n_fe; a++) {
                h_rid[go + a] = (int)k;
                h_orig[go + a] = r->ge_idx[a];
            }
            for (int64_t b = 0; b < r->n_fe; b += 256) h_chunks.push_back({(int)k, (int)(fo + b), (int)std::min<int64_t>(fo + r->n_fe, fo + b + 256)});
            for (int64_t b = 0; b < r->n - r->n_fe; b += 256)
                h_chunks.push_back({(int)k, (int)(go + b), (int)std::min<int64_t>(go + r->n - r->n_fe, go + b + 256)});
            cmax = std::max(cmax, r->ncol);
            fo += (int)r->n_fe;
            go += (int)(r->n - r->n_fe);
            h_rep[k] = r->dev;
            h_rep[k].landau_a = M ? M->landau[0] : 0.0;   // the model's term, read by the spin kernels
            h_rep[k].landau_b = M ? M->landau[1] : 0.0;
        }
        h_cptr.push_back((int)h_chunks.size());
        n_cells = cb;
        n_chunks = (int)h_chunks.size();
        // colour classes
        // (counting sort: inside a colour, replica order, then atom order)
        col_ptr.assign(cmax + 1, 0);
        for (Replica *r : reps)
            for (int c : r->colour_fe) col_ptr[c + 1]++;
        for (int c = 0; c < cmax; c++) col_ptr[c + 1] += col_ptr[c];
        std::vector<int> h_colidx(col_ptr[cmax]);
        {
            std::vector<int> fill(col_ptr.begin(), col_ptr.end() - 1);
            for (Replica *r : reps)
                for (int64_t a = 0; a < (int64_t)r->colour_fe.size(); a++)
                    h_colidx[fill[r->colour_fe[a]]++] = r->fe_off + (int)a;
        }
        // spin carriers without a colour (evaluation only) keep their own index
        std::vector<int> h_colpos(nfe);
        for (size_t q = 0; q < nfe; q++) h_colpos[q] = (int)q;
        if (h_colidx.size() == nfe)
            for (size_t q = 0; q < nfe; q++) h_colpos[h_colidx[q]] = (int)q;
        if (nfe) HIPCHK(hipMemcpyAsync(colpos, h_colpos.data(), nfe * 4, hipMemcpyHostToDevice, st));
        if (n) {
            HIPCHK(hipMemcpyAsync(rid, h_rid.data(), n * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(orig, h_orig.data(), n * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(colour, h_col.data(), n * 4, hipMemcpyHostToDevice, st));
        }
        if (!h_rep.empty()) HIPCHK(hipMemcpyAsync(rep, h_rep.data(), h_rep.size() * sizeof(RepDev), hipMemcpyHostToDevice, st));
        if (!h_chunks.empty()) HIPCHK(hipMemcpyAsync(chunks, h_chunks.data(), h_chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(chunk_ptr, h_cptr.data(), h_cptr.size() * 4, hipMemcpyHostToDevice, st));
        std::vector<int> h_colrid(h_colidx.size());
        for (size_t q = 0; q < h_colidx.size(); q++) h_colrid[q] = h_rid[h_colidx[q]];
        if (!h_colidx.empty()) {
            HIPCHK(hipMemcpyAsync(col_idx, h_colidx.data(), h_colidx.size() * 4, hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(col_rid, h_colrid.data(), h_colrid.size() * 4, hipMemcpyHostToDevice, st));
        }
        // state: the kept replicas' rows from the staging buffer in one gather
        if (stage && n) {
            if (n > src_cap) {
                if (src_buf) (void)hipFree(src_buf);
                src_buf = nullptr;
                src_cap = 0;
                if (hipMalloc((void **)&src_buf, n * sizeof(int)) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(SL_E_OOM, "hipMalloc of the re-layout index failed");
                }
                src_cap = n;
            }
            std::vector<int> h_src(n, -1);
            for (size_t m = 0; m < moved.size(); m++) {
                const Replica *r = moved[m];
                for (int64_t q = 0; q < r->n_fe; q++) h_src[r->fe_off + q] = old_fe[m] + (int)q;
                for (int64_t q = 0; q < r->n - r->n_fe; q++) h_src[r->ge_off + q] = old_ge[m] + (int)q;
            }
            HIPCHK(hipMemcpyAsync(src_buf, h_src.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
            launch_gather_state(stage, n_old, src_buf, (int)n, pos, vel, spin, force, field, st);
            HIPCHK(hipStreamSynchronize(st));
        }
        std::vector<d4> buf;
        for (size_t k = 0; k < reps.size(); k++) {
            Replica *r = reps[k];
            auto mk = std::find(moved.begin(), moved.end(), r);
            d4 *dst[5] = {pos, vel, spin, force, field};
            if (mk != moved.end()) {
                if (stage) continue;   // gathered above
                size_t m = mk - moved.begin();
                for (int a = 0; a < 5; a++) {
                    const d4 *from = snap[5 * m + a].data();
                    if (r->n_fe)
                        HIPCHK(hipMemcpyAsync(dst[a] + r->fe_off, from, r->n_fe * sizeof(d4), hipMemcpyHostToDevice,
                                              st));
                    if (r->n - r->n_fe)
                        HIPCHK(hipMemcpyAsync(dst[a] + r->ge_off, from + r->n_fe, (r->n - r->n_fe) * sizeof(d4),
                                              hipMemcpyHostToDevice, st));
                }
            } else {
                const double *src[3] = {r->pos.data(), r->vel.data(), r->spin.data()};
                for (int a = 0; a < 3; a++) {
                    buf.assign(r->n, d4{0, 0, 0, 0});
                    for (int64_t q = 0; q < r->n_fe; q++) {
                        const int c = r->fe_idx[q];
                        buf[q] = d4{src[a][3 * c], src[a][3 * c + 1], src[a][3 * c + 2], 0.0};
                    }
                    for (int64_t q = 0; q < r->n - r->n_fe; q++) {
                        const int c = r->ge_idx[q];
                        if (a == 2) buf[r->n_fe + q] = d4{0, 0, 0, 0};   // no spin on species 1
                        else buf[r->n_fe + q] = d4{src[a][3 * c], src[a][3 * c + 1], src[a][3 * c + 2], 0.0};
                    }
                    if (r->n_fe)
                        HIPCHK(hipMemcpyAsync(dst[a] + r->fe_off, buf.data(), r->n_fe * sizeof(d4), hipMemcpyHostToDevice, st));
                    if (r->n - r->n_fe)
                        HIPCHK(hipMemcpyAsync(dst[a] + r->ge_off, buf.data() + r->n_fe, (r->n - r->n_fe) * sizeof(d4),
                                              hipMemcpyHostToDevice, st));
                    HIPCHK(hipStreamSynchronize(st));
                }
            }
        }
        if (stage) HIPCHK(hipStreamSynchronize(st));
        // clear the error flags, force a neighbour rebuild, then F and H
        int hflags[NFLAGS] = {0};
        hflags[F_REBUILD] = 1;
        HIPCHK(hipMemcpyAsync(flags, hflags, sizeof(hflags), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        if (N) {
            const Sys S = sys();
            launch_rebuild(S, RC_R + max_skin(), RC_A + max_skin(), st);
            // Replicas carried over from the previous layout keep their forces
            // and fields: neighbour order inside a replica does not depend on
            // where the replica sits, so an evaluation here would reproduce
            // them bitwise. Only the replicas new to the device are evaluated,
            // the others being marked inactive meanwhile.
            if (moved.empty()) {
                evaluate(spin);
            } else if (moved.size() < reps.size()) {
                // only the 'active' words change: the rebuild may have set
                // failure bits in the replica records, which must survive
                std::vector<int> off(reps.size(), -1), back(reps.size(), -1);
                for (Replica *r : moved) {
                    off[r->slot] = 0;
                    back[r->slot] = h_rep[r->slot].active;
                }
                HIPCHK(hipMemcpyAsync(act_buf, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, st));
                launch_set_active(rep, act_buf, (int)reps.size(), st);
                evaluate(spin);
                HIPCHK(hipMemcpyAsync(act_buf + reps.size(), back.data(), back.size() * sizeof(int),
                                      hipMemcpyHostToDevice, st));
                launch_set_active(rep, act_buf + reps.size(), (int)reps.size(), st);
                HIPCHK(hipStreamSynchronize(st));
            }
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return SL_OK;
    }

    double max_skin() const {
        double s = 0;
        for (Replica *r : reps) s = std::max(s, r->dev.skin);
        return s;
    }

    // forward + backward at the current positions and the given spins
    template <typename real>
    void forward(const ModelDev<real> &m, const Work<real> &w, const d4 *spins, int mode = PASS_FULL) {
        const Sys S = sys();
        { ProfScope p(this, 0); launch_desc_radial(S, m, w, spins, mode, st); }
        { ProfScope p(this, 1); launch_desc_angular(S, m, w, spins, mode, st); }
        { ProfScope p(this, 2); launch_mlp(S, m, w, mode, st); }
    }

    template <typename real>
    void backward(const ModelDev<real> &m, const Work<real> &w) {
        const Sys S = sys();
        { ProfScope p(this, 3); launch_bwd_radial(S, m, w, st); }
        { ProfScope p(this, 4); launch_bwd_angular(S, m, w, 0, st); }
        { ProfScope p(this, 11); launch_bwd_angular(S, m, w, 1, st); }
        { ProfScope p(this, 5); launch_gather(S, w, st); }
    }

    void evaluate(const d4 *spins) {
        if (prec == SL_FP64) {
            forward(M->m64, w64, spins);
            backward(M->m64, w64);
        } else {
            forward(M->m32, w32, spins);
            backward(M->m32, w32);
        }
    }

    void rebuild_if_needed() {
        ProfScope p(this, 8);
        const Sys S = sys();
        launch_skin_check(S, st);
        launch_rebuild(S, RC_R + max_skin(), RC_A + max_skin(), st);
    }

    template <typename real>
    void spin_step(const ModelDev<real> &m, const Work<real> &w) {
        const Sys S = sys();
        { ProfScope q(this, 9); launch_spin_prep(S, st); }
        // iterated to a tolerance when any replica asks for it (each stops on
        // its own criterion; the others after their K_corr correctors)
        bool sc = false;
        int cap = 0;
        for (const Replica *r : reps)
            if (r->dev.sc_tol > 0) {
                sc = true;
                cap = std::max(cap, r->dev.sc_max);
            }
        const int last = sc ? std::max(cap, K_corr) : K_corr;
        int passes = 0;
        double change = 0;
        for (int p = 0; p <= last; p++) {
            // every pass sits at the same mid positions: the structural terms of the first are reused
            forward(m, w, spin_hat, p == 0 ? PASS_SPIN : PASS_SPIN_REUSE);
            { ProfScope q(this, 6); launch_assemble_coef(S, m, w, st); }
            { ProfScope q(this, 10); launch_assemble_pairs(S, m, w, st); }
            if (p > 0) {
                ProfScope q(this, 9);
                launch_spin_restore(S, st);
            }
            {
                ProfScope q(this, 7);
                launch_sweep(S, w, col_ptr.data(), (int)col_ptr.size() - 1, st);
            }
            passes = p + 1;
            if (sc) {
                // the host waits for the decision: one small read per pass
                double out[2] = {0, 0};
                {
                    ProfScope q(this, 9);
                    launch_sc_check(S, p, sc_depth, sc_reg, K_corr, st);
                }
                if (hipMemcpyAsync(out, sc_out, sizeof(out), hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    out[0] = 0;   // the step's own error checks report the failure
                change = out[1];
                if (out[0] == 0) break;
            }
            if (p < last) {
                ProfScope q(this, 9);
                if (sc && sc_depth > 0) launch_sc_mix(S, p, sc_depth, st);
                else launch_spin_mid(S, st);
            }
        }
        if (sc) {
            log_passes.push_back(passes);
            log_change.push_back(change);
        }
    }

    // one B A O S A B step of every active replica; observables to obs_out[n_rep][NOBS]
    void step(double *obs_out) {
        const Sys S = sys();
        { ProfScope p(this, 9); launch_kick(S, st); launch_drift(S, st); }
        rebuild_if_needed();
        { ProfScope p(this, 9); launch_langevin(S, st); }
        if (!M->structural) {
            if (prec == SL_FP64) spin_step(M->m64, w64);
            else spin_step(M->m32, w32);
        }
        { ProfScope p(this, 9); launch_drift(S, st); }
        rebuild_if_needed();
        evaluate(spin);
        ProfScope p(this, 9);
        launch_kick(S, st);
        if (prec == SL_FP64) launch_observe(S, w64, chunks, n_chunks, chunk_ptr, partial, obs_out, st);
        else launch_observe(S, w32, chunks, n_chunks, chunk_ptr, partial, obs_out, st);
        launch_step_end(S, st);
    }

    int read_flags(int *h) {
        HIPCHK(hipMemcpyAsync(h, flags, NFLAGS * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return SL_OK;
    }

    int check_flags() {
        int h[NFLAGS];
        int rc = read_flags(h);
        if (rc) return rc;
        if (h[F_OVERFLOW] & 1) return fail(SL_E_OVERFLOW, "neighbour list capacity exceeded (more than 160 atoms within rc_R+skin, 96 within rc_A+skin or 64 spin neighbours)");
        if (h[F_OVERFLOW] & 2) return fail(SL_E_OVERFLOW, "asymmetric neighbour lists");
        return SL_OK;
    }

    // device records of the resident replicas (step counters, failure bits)
    int read_reps(std::vector<RepDev> &out) {
        out.resize(reps.size());
        if (!reps.empty())
            HIPCHK(hipMemcpyAsync(out.data(), rep, reps.size() * sizeof(RepDev), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return SL_OK;
    }
    int write_rep(const Replica *r, const RepDev &d) {
        HIPCHK(hipMemcpyAsync(rep + r->slot, &d, sizeof(RepDev), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return SL_OK;
    }

    // state of replica r in caller order
    int download(Replica *r, double *p, double *v, double *s) {
        d4 *src[3] = {pos, vel, spin};
        double *dst[3] = {p, v, s};
        std::vector<d4> buf(r->n);
        for (int a = 0; a < 3; a++) {
            if (!dst[a]) continue;
            if (r->n_fe) HIPCHK(hipMemcpyAsync(buf.data(), src[a] + r->fe_off, r->n_fe * sizeof(d4), hipMemcpyDeviceToHost, st));
            if (r->n - r->n_fe)
                HIPCHK(hipMemcpyAsync(buf.data() + r->n_fe, src[a] + r->ge_off, (r->n - r->n_fe) * sizeof(d4),
                                      hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t q = 0; q < r->n; q++) {
                const int c = q < r->n_fe ? r->fe_idx[q] : r->ge_idx[q - r->n_fe];
                dst[a][3 * c] = buf[q].x;
                dst[a][3 * c + 1] = buf[q].y;
                dst[a][3 * c + 2] = buf[q].z;
            }
        }
        return SL_OK;
    }

    int download_ff(Replica *r, double *F, double *H) {
        d4 *src[2] = {force, field};
        double *dst[2] = {F, H};
        std::vector<d4> buf(r->n);
        for (int a = 0; a < 2; a++) {
            if (!dst[a]) continue;
            if (r->n_fe) HIPCHK(hipMemcpyAsync(buf.data(), src[a] + r->fe_off, r->n_fe * sizeof(d4), hipMemcpyDeviceToHost, st));
            if (r->n - r->n_fe)
                HIPCHK(hipMemcpyAsync(buf.data() + r->n_fe, src[a] + r->ge_off, (r->n - r->n_fe) * sizeof(d4),
                                      hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t q = 0; q < r->n; q++) {
                const int c = q < r->n_fe ? r->fe_idx[q] : r->ge_idx[q - r->n_fe];
                dst[a][3 * c] = buf[q].x;
                dst[a][3 * c + 1] = buf[q].y;
                dst[a][3 * c + 2] = buf[q].z;
            }
        }
        return SL_OK;
    }

    template <typename real>
    int download_rows(Replica *r, const real *src, int width, int stride, double *dst) {
        std::vector<real> buf((size_t)r->n * stride);
        if (r->n_fe)
            HIPCHK(hipMemcpyAsync(buf.data(), src + (size_t)r->fe_off * stride, (size_t)r->n_fe * stride * sizeof(real),
                                  hipMemcpyDeviceToHost, st));
        if (r->n - r->n_fe)
            HIPCHK(hipMemcpyAsync(buf.data() + (size_t)r->n_fe * stride, src + (size_t)r->ge_off * stride,
                                  (size_t)(r->n - r->n_fe) * stride * sizeof(real), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t q = 0; q < r->n; q++) {
            const int c = q < r->n_fe ? r->fe_idx[q] : r->ge_idx[q - r->n_fe];
            for (int k = 0; k < width; k++) dst[(size_t)c * width + k] = (double)buf[(size_t)q * stride + k];
        }
        return SL_OK;
    }
};

// ---------------------------------------------------------------------------
// replica construction and validation
// ---------------------------------------------------------------------------

static int check_view(const sl_system_view *sys, double skin) {
    if (!sys || sys->n_atoms < 0 || (sys->n_atoms > 0 && (!sys->types || !sys->pos)))
        return fail(SL_E_INVALID, "system view: missing arrays");
    if (sys->n_atoms > INT_MAX / 2) return fail(SL_E_INVALID, "too many atoms");
    for (int64_t i = 0; i < sys->n_atoms; i++)
        if (sys->types[i] != 0 && sys->types[i] != 1) return fail(SL_E_INVALID, "species must be 0 or 1");
    for (int a = 0; a < 3; a++) {
        if (!(sys->box[a] > 0) && sys->pbc[a]) return fail(SL_E_BOX, "periodic box edge must be positive");
        if (sys->pbc[a] && sys->box[a] < 2.0 * (RC_R + skin))
            return fail(SL_E_BOX, "periodic box edge shorter than 2 (rc_R + skin)");
    }
    for (int64_t i = 0; i < 3 * sys->n_atoms; i++)
        if (!std::isfinite(sys->pos[i]) || (sys->spin && !std::isfinite(sys->spin[i])))
            return fail(SL_E_INVALID, "non-finite position or spin");
    return SL_OK;
}

// greedy colouring of the spin carriers (graph: r < rc_R + skin + 0.5), in
// index order; with `keep` a repair: a spin keeps its colour unless a
// neighbour has it, and then takes the smallest colour no neighbour has.
// A repaired spin takes a colour none of its neighbours has, so a repair never
// creates a conflict: only spins that share their colour with a neighbour at
// the start can change, and they are found by looking at same-colour spins
// alone (cells per colour), then repaired in index order.
static int greedy_colour(const sl_system_view *sys, double skin, std::vector<int> &col,
                         const std::vector<int> *keep = nullptr) {
    const int64_t n = sys->n_atoms;
    if (keep) col = *keep;
    else col.assign(n, -1);
    const double rc = RC_R + skin + 0.5, rc2 = rc * rc;
    std::vector<int> fe;
    for (int64_t i = 0; i < n; i++)
        if (sys->types[i] == 0) fe.push_back((int)i);
    // bin spin carriers
    int nc[3];
    double lo[3], w[3], ib[3];
    for (int a = 0; a < 3; a++) {
        double mn = 1e300, mx = -1e300;
        ib[a] = sys->pbc[a] ? 1.0 / sys->box[a] : 0.0;
        for (int i : fe) {
            double x = sys->pos[3 * i + a];
            if (sys->pbc[a]) x -= sys->box[a] * std::floor(x * ib[a]);
            mn = std::min(mn, x);
            mx = std::max(mx, x);
        }
        if (sys->pbc[a]) {
            lo[a] = 0;
            nc[a] = std::max(1, (int)std::floor(sys->box[a] / rc));
            w[a] = sys->box[a] / nc[a];
        } else {
            lo[a] = mn - 1;
            double ext = mx - mn + 2;
            nc[a] = std::max(1, (int)std::floor(ext / rc));
            w[a] = ext / nc[a];
        }
        if (nc[a] > 1024) return fail(SL_E_INVALID, "colouring grid too large");
    }
    const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
    std::vector<int> cid(n, -1);
    for (int i : fe) {
        int c[3];
        for (int a = 0; a < 3; a++) {
            double x = sys->pos[3 * i + a] - lo[a];
            if (sys->pbc[a]) x -= sys->box[a] * std::floor(x * ib[a]);
            c[a] = std::min(nc[a] - 1, std::max(0, (int)std::floor(x / w[a])));
        }
        cid[i] = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
    }
    auto dist2 = [&](int i, int j) {
        double d2 = 0;
        for (int a = 0; a < 3; a++) {
            double x = sys->pos[3 * j + a] - sys->pos[3 * i + a];
            if (sys->pbc[a]) x -= sys->box[a] * std::nearbyint(x * ib[a]);
            d2 += x * x;
        }
        return d2;
    };
    // the 27 cells around a cell (fewer on free axes; periodic images folded)
    auto around = [&](size_t ci, int out[27]) {
        const int c0 = (int)(ci / ((size_t)nc[1] * nc[2])), c1 = (int)((ci / nc[2]) % nc[1]), c2 = (int)(ci % nc[2]);
        int k = 0;
        for (int dx = -1; dx <= 1; dx++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dz = -1; dz <= 1; dz++) {
                    int cc[3] = {c0 + dx, c1 + dy, c2 + dz};
                    bool ok = true;
                    for (int a = 0; a < 3; a++) {
                        if (cc[a] < 0 || cc[a] >= nc[a]) {
                            if (sys->pbc[a]) cc[a] = (cc[a] + nc[a]) % nc[a];
                            else ok = false;
                        }
                    }
                    if (!ok) continue;
                    const int v = (cc[0] * nc[1] + cc[1]) * nc[2] + cc[2];
                    bool dup = false;   // small periodic grids fold onto the same cell
                    for (int q = 0; q < k; q++) dup |= out[q] == v;
                    if (!dup) out[k++] = v;
                }
        return k;
    };
    // spin carriers by cell (counting sort)
    std::vector<int> start(ncell + 1, 0), members(fe.size());
    for (int i : fe) start[cid[i] + 1]++;
    for (size_t c = 0; c < ncell; c++) start[c + 1] += start[c];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int i : fe) members[fill[cid[i]]++] = i;
    }
    std::vector<char> used(512, 0);
    auto pick = [&](int i) {   // smallest colour none of i's neighbours has; col[i] if that one is free
        std::fill(used.begin(), used.end(), 0);
        int cells[27];
        const int k = around(cid[i], cells);
        for (int q = 0; q < k; q++)
            for (int m = start[cells[q]]; m < start[cells[q] + 1]; m++) {
                const int j = members[m];
                if (j != i && col[j] >= 0 && col[j] < (int)used.size() && dist2(i, j) < rc2) used[col[j]] = 1;
            }
        if (col[i] >= 0 && col[i] < (int)used.size() && !used[col[i]]) return col[i];
        int c = 0;
        while (c < (int)used.size() && used[c]) c++;
        return c;
    };
    if (!keep) {
        for (int i : fe) col[i] = pick(i);
        return SL_OK;
    }
    // spins that share their colour with a neighbour: cells per colour
    int ncol = 0;
    for (int i : fe) ncol = std::max(ncol, col[i] + 1);
    std::vector<int> cstart((size_t)ncol * ncell + 1, 0), cmem(fe.size());
    for (int i : fe)
        if (col[i] >= 0) cstart[(size_t)col[i] * ncell + cid[i] + 1]++;
    for (size_t c = 0; c < (size_t)ncol * ncell; c++) cstart[c + 1] += cstart[c];
    {
        std::vector<int> fill(cstart.begin(), cstart.end() - 1);
        for (int i : fe)
            if (col[i] >= 0) cmem[fill[(size_t)col[i] * ncell + cid[i]]++] = i;
    }
    std::vector<int> flagged;
    for (int i : fe) {
        if (col[i] < 0) {
            flagged.push_back(i);
            continue;
        }
        int cells[27];
        const int k = around(cid[i], cells);
        bool hit = false;
        for (int q = 0; q < k && !hit; q++) {
            const size_t b = (size_t)col[i] * ncell + cells[q];
            for (int m = cstart[b]; m < cstart[b + 1] && !hit; m++) {
                const int j = cmem[m];
                hit = j != i && dist2(i, j) < rc2;
            }
        }
        if (hit) flagged.push_back(i);
    }
    for (int i : flagged) col[i] = pick(i);
    return SL_OK;
}

// Repaired colouring of a resident replica from its current positions; the
// pause bit is cleared and the replica re-activated. The caller re-lays out.
static int recolour_replica(Engine &e, Replica *r) {
    std::vector<double> p(3 * r->n);
    int rc = e.download(r, p.data(), nullptr, nullptr);
    if (rc) return rc;
    std::vector<int32_t> types(r->n, 1);
    for (int q : r->fe_idx) types[q] = 0;
    sl_system_view v{};
    v.n_atoms = r->n;
    v.types = types.data();
    v.pos = p.data();
    for (int a = 0; a < 3; a++) {
        v.box[a] = r->dev.box[a];
        v.pbc[a] = r->dev.pbc[a];
    }
    // repair the present colouring: only spins that now meet their colour
    // inside the colouring radius change
    std::vector<int> col(r->n, -1);
    for (int64_t q = 0; q < r->n_fe; q++) col[r->fe_idx[q]] = r->colour_fe[q];
    const std::vector<int> prev = col;
    if ((rc = greedy_colour(&v, r->dev.skin, col, &prev))) return rc;
    r->ncol = 0;
    for (int64_t q = 0; q < r->n_fe; q++) {
        r->colour_fe[q] = col[r->fe_idx[q]];
        r->ncol = std::max(r->ncol, r->colour_fe[q] + 1);
    }
    std::vector<RepDev> d;
    if ((rc = e.read_reps(d))) return rc;
    RepDev x = d[r->slot];
    x.failed &= ~4;
    x.active = x.step < x.step_end;
    r->n_recolour++;
    return e.write_rep(r, x);
}

// After a (re)layout: turn the replicas' failure bits into errors, recolour
// those whose colouring conflicts inside the list shell, and lay out again.
// bad[k] receives the status of replica k (SL_OK if it may run).
static int settle_layout(Engine &e, std::vector<int> &bad, bool global_flags = true) {
    for (int it = 0; it < 4; it++) {
        int rc = global_flags ? e.check_flags() : SL_OK;
        if (rc) return rc;
        std::vector<RepDev> d;
        if ((rc = e.read_reps(d))) return rc;
        bad.assign(d.size(), SL_OK);
        bool again = false;
        for (size_t k = 0; k < d.size(); k++) {
            if (d[k].failed & 1) bad[k] = SL_E_OVERFLOW;
            else if (d[k].failed & 2) bad[k] = SL_E_INVALID;
            else if (d[k].failed & 4) {
                if ((rc = recolour_replica(e, e.reps[k]))) return rc;
                again = true;
            }
        }
        if (!again) return SL_OK;
        std::vector<Replica *> same = e.reps;
        if ((rc = e.set_layout(same))) return rc;
    }
    return fail(SL_E_INVALID, "recolouring did not settle");
}

// largest replica whose spin carriers are stored colour by colour
constexpr int64_t COLOUR_MAJOR_MAX_ATOMS = 1 << 19;

static const char *colour_msg = "two spins of the same colour lie within rc_R of each other (invalid colouring)";

static int make_replica(const sl_system_view *sys, const double *vel, const int32_t *colour,
                        const sl_integrator_params *ip, bool need_colour, Replica &r, bool structural = false) {
    const double skin = ip ? ip->skin : 0.5;
    if (ip && !(ip->skin >= 0 && ip->skin < 5)) return fail(SL_E_INVALID, "skin must be in [0, 5)");
    int rc = check_view(sys, skin);
    if (rc) return rc;
    const int64_t n = sys->n_atoms;
    r.n = n;
    r.fe_idx.clear();
    r.ge_idx.clear();
    for (int64_t i = 0; i < n; i++) (sys->types[i] == 0 ? r.fe_idx : r.ge_idx).push_back((int)i);
    r.n_fe = (int64_t)r.fe_idx.size();
    r.pos.assign(sys->pos, sys->pos + 3 * n);
    r.vel.assign(3 * n, 0.0);
    if (vel) r.vel.assign(vel, vel + 3 * n);
    r.spin.assign(3 * n, 0.0);
    if (sys->spin && !structural) r.spin.assign(sys->spin, sys->spin + 3 * n);
    for (int64_t i = 0; i < n; i++)
        if (sys->types[i] != 0) r.spin[3 * i] = r.spin[3 * i + 1] = r.spin[3 * i + 2] = 0.0;
    RepDev &d = r.dev;
    std::memset(&d, 0, sizeof(d));
    for (int a = 0; a < 3; a++) {
        d.box[a] = sys->box[a];
        d.ibox[a] = sys->box[a] > 0 ? 1.0 / sys->box[a] : 0.0;
        d.pbc[a] = sys->pbc[a] ? 1 : 0;
        d.B0[a] = d.B1[a] = sys->B[a];
    }
    d.mu_s = sys->mu_s;
    d.skin = skin;
    d.active = 1;
    d.step_end = LLONG_MAX;
    d.mass[0] = mass_of(0);
    d.mass[1] = mass_of(1);
    if (ip) {
        for (int t = 0; t < 2; t++) {
            if (!(ip->mass[t] >= 0 && std::isfinite(ip->mass[t]))) return fail(SL_E_INVALID, "masses must be >= 0");
            if (ip->mass[t] > 0) d.mass[t] = ip->mass[t];
        }
        if (!(ip->dt != 0 && std::isfinite(ip->dt))) return fail(SL_E_INVALID, "dt must be finite and non-zero");
        if (ip->mid_cap < 1 || ip->mid_cap > 1000) return fail(SL_E_INVALID, "mid_cap must be in [1, 1000]");
        if (ip->K_corr < 0 || ip->K_corr > 64) return fail(SL_E_INVALID, "K_corr must be in [0, 64]");
        if (!(ip->sc_tol >= 0 && std::isfinite(ip->sc_tol))) return fail(SL_E_INVALID, "sc_tol must be finite, >= 0");
        if (ip->sc_tol > 0 && (ip->sc_max < 1 || ip->sc_max > 1000))
            return fail(SL_E_INVALID, "sc_max must be in [1, 1000]");
        if (ip->sc_tol > 0 && (ip->sc_depth < 0 || ip->sc_depth > SC_MAXD || !(ip->sc_reg >= 0) ||
                               !std::isfinite(ip->sc_reg)))
            return fail(SL_E_INVALID, "sc_depth must be in [0, 8] and sc_reg finite and >= 0");
        if (ip->alpha_s < 0 || ip->T0 < 0 || ip->T1 < 0 || ip->gamma_L < 0)
            return fail(SL_E_INVALID, "alpha_s, temperatures and gamma_L must be non-negative");
        if (ip->longitudinal != 0 && ip->longitudinal != 1) return fail(SL_E_INVALID, "longitudinal must be 0 or 1");
        if (!(ip->gamma_lsf >= 0 && std::isfinite(ip->gamma_lsf)))
            return fail(SL_E_INVALID, "gamma_lsf must be finite and >= 0");
        if (ip->longitudinal && ip->alpha_s != 0)
            return fail(SL_E_INVALID, "with longitudinal = 1 the damping is gamma_lsf: alpha_s must be 0");
        d.lsf = ip->longitudinal;
        d.lsf_gamma = ip->longitudinal ? ip->gamma_lsf : 0.0;
        d.dt = ip->dt;
        d.T0 = ip->T0;
        d.T1 = ip->T1;
        d.alpha = ip->alpha_s;
        d.gammaL = ip->gamma_L;
        d.mid_tol = ip->mid_tol;
        d.mid_cap = ip->mid_cap;
        d.sc_tol = ip->sc_tol;
        d.sc_max = ip->sc_max;
        d.n_ramp = ip->n_ramp;
        d.seed = ip->seed;
        d.ensemble = ip->ensemble;
        for (int a = 0; a < 3; a++) {
            d.B0[a] = ip->B0[a];
            d.B1[a] = ip->B1[a];
        }
    }
    Engine::cell_grid(r, sys->pos);
    if (need_colour) {
        std::vector<int> col;
        if (colour) {
            col.assign(colour, colour + n);
        } else {
            rc = greedy_colour(sys, skin, col);
            if (rc) return rc;
        }
        for (int64_t q = 0; q < r.n_fe; q++) {
            const int c = col[r.fe_idx[q]];
            if (c < 0 || c > 4096) return fail(SL_E_INVALID, "colour of a spin carrier must be in [0, 4096]");
        }
        // Replicas whose gathered per-atom data (about 0.4 KB per atom) fits
        // in the 256 MB last-level cache store their spin carriers colour by
        // colour (caller order inside a colour): a colour class is then a
        // contiguous run of atoms, so the coupling assembly, which writes each
        // spin's couplings at its colour-list position, stores contiguously,
        // and the sweep reads contiguously. Larger ones keep the caller
        // order, whose spatial locality the neighbour gathers need once the
        // system no longer fits in that cache.
        if (n <= COLOUR_MAJOR_MAX_ATOMS)
            std::stable_sort(r.fe_idx.begin(), r.fe_idx.end(), [&](int a, int b) { return col[a] < col[b]; });
        r.colour_fe.resize(r.n_fe);
        r.ncol = 0;
        for (int64_t q = 0; q < r.n_fe; q++) {
            const int c = col[r.fe_idx[q]];
            r.colour_fe[q] = c;
            r.ncol = std::max(r.ncol, c + 1);
        }
    }
    return SL_OK;
}

// ---------------------------------------------------------------------------
// model API
// ---------------------------------------------------------------------------

// The structural-only model in the spin-aware layout: its radial and angular
// coefficients, zero magnetic coefficients, and per species W0 with zero
// columns for the magnetic channels; with no spins both define one energy.
static std::vector<double> expand_structural(const double *p) {
    std::vector<double> out(N_PARAMS, 0.0);
    std::copy(p, p + P_CEX, out.begin());   // c^R, c^A
    size_t src = P_CEX, dst = P_MLP;
    for (int t = 0; t < 2; t++) {
        for (int h = 0; h < NH; h++)
            for (int d = 0; d < DS; d++) out[dst + (size_t)h * ND + d] = p[src + (size_t)h * DS + d];
        src += (size_t)NH * DS;
        dst += (size_t)NH * ND;
        for (int k = 0; k < 2 * NH + 1; k++) out[dst + k] = p[src + k];   // b0, w1, b1
        src += 2 * NH + 1;
        dst += 2 * NH + 1;
    }
    return out;
}

extern "C" int nep_model_create(const nep_spin_hparams *hp, const double *params, size_t n_params,
                                nep_model **out) {
    if (!out) return fail(SL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!hp || !params) return fail(SL_E_INVALID, "hparams and params are required");
    if (hp->n_max_R != 8 || hp->n_max_A != 6 || hp->l_max != 4 || hp->basis_K != 8 || hp->n_hidden != 64 ||
        hp->n_species != 2 || hp->rc_R != RC_R || hp->rc_A != RC_A)
        return fail(SL_E_INVALID, "unsupported hyper-parameters (supported: n_max_R 8, n_max_A 6, l_max 4, "
                                  "basis_K 8, n_hidden 64, 2 species, rc 6.0/4.5)");
    if (hp->structural != 0 && hp->structural != 1) return fail(SL_E_INVALID, "structural must be 0 or 1");
    if (!std::isfinite(hp->moment_a) || !std::isfinite(hp->moment_b) || hp->moment_b < 0)
        return fail(SL_E_INVALID, "moment-length term: moment_a, moment_b must be finite and moment_b >= 0");
    if (hp->sr_r_outer != 0.0) {
        const bool ok = std::isfinite(hp->sr_Z[0]) && std::isfinite(hp->sr_Z[1]) && hp->sr_Z[0] > 0 &&
                        hp->sr_Z[1] > 0 && std::isfinite(hp->sr_r_inner) && hp->sr_r_inner > 0 &&
                        hp->sr_r_inner < hp->sr_r_outer && hp->sr_r_outer <= RC_R;
        if (!ok)
            return fail(SL_E_INVALID, "short-range term: need Z_0, Z_1 > 0 and 0 < r_inner < r_outer <= rc_R "
                                      "(r_outer = 0 turns it off)");
    }
    const size_t want = hp->structural ? (size_t)N_PARAMS_STRUCT : (size_t)N_PARAMS;
    if (n_params != want)
        return fail(SL_E_INVALID, hp->structural ? "expected 5570 parameters (structural-only model)"
                                                 : "expected 15438 parameters");
    for (size_t k = 0; k < n_params; k++)
        if (!std::isfinite(params[k])) return fail(SL_E_INVALID, "non-finite parameter");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(SL_E_NOLIB, "no HIP device");
    }
    auto m = std::make_unique<nep_model>();
    m->structural = hp->structural == 1;
    if (hp->sr_r_outer != 0.0) {
        m->zbl[0] = hp->sr_Z[0];
        m->zbl[1] = hp->sr_Z[1];
        m->zbl[2] = hp->sr_r_inner;
        m->zbl[3] = hp->sr_r_outer;
    }
    if (!m->structural) {
        m->landau[0] = hp->moment_a;
        m->landau[1] = hp->moment_b;
    }
    if (m->structural) m->p = expand_structural(params);
    else m->p.assign(params, params + n_params);
    std::vector<double> h64;
    std::vector<float> h32;
    model_layout(m->p, m->zbl, h64);
    model_layout(m->p, m->zbl, h32);
    int rc;
    if ((rc = dalloc(&m->d64, MODEL_DEV)) || (rc = dalloc(&m->d32, MODEL_DEV))) return rc;
    HIPCHK(hipMemcpy(m->d64, h64.data(), MODEL_DEV * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(m->d32, h32.data(), MODEL_DEV * 4, hipMemcpyHostToDevice));
    m->m64 = model_ptrs(m->d64);
    m->m32 = model_ptrs(m->d32);
    *out = m.release();
    return SL_OK;
}

extern "C" int nep_model_destroy(nep_model *m) {
    if (!m) return SL_OK;
    for (auto &e : m->eval_eng) delete e;
    dfree(m->d64);
    dfree(m->d32);
    delete m;
    return SL_OK;
}

static int check_prec(sl_precision p) {
    if (p != SL_FP64 && p != SL_FP32_MIXED)
        return fail(SL_E_INVALID, "unknown precision (SL_FP64 or SL_FP32_MIXED)");
    return SL_OK;
}

// evaluation of one system on the model's cached engine
static int eval_common(const nep_model *mc, const sl_system_view *sys, sl_precision prec, Replica &r,
                       Engine *&eng) {
    nep_model *m = const_cast<nep_model *>(mc);
    int rc = check_prec(prec);
    if (rc) return rc;
    if ((rc = make_replica(sys, nullptr, nullptr, nullptr, false, r, m->structural))) return rc;
    // one evaluation engine per model: the work arrays of another precision,
    // or of a system more than eight times larger, are released first
    for (int q = 0; q < 2; q++)
        if (m->eval_eng[q] && (q != (int)prec || (size_t)r.n * 8 < m->eval_eng[q]->cap)) {
            delete m->eval_eng[q];
            m->eval_eng[q] = nullptr;
        }
    Engine *&e = m->eval_eng[prec];
    if (!e) {
        e = new Engine();
        e->M = m;
        e->prec = prec;
    }
    eng = e;
    e->reps.clear();   // the previous call's replica no longer exists
    if ((rc = e->set_layout({&r}))) return rc;
    return e->check_flags();
}

// an empty system: zero energy, nothing else written
static int eval_empty(sl_precision prec, double *energy, const sl_exec *ex) {
    int rc = check_prec(prec);
    if (rc) return rc;
    const double z = 0.0;
    if (energy) {
        if (ex && ex->device_ptrs) HIPCHK(hipMemcpy(energy, &z, 8, hipMemcpyHostToDevice));
        else *energy = 0.0;
    }
    return SL_OK;
}

// E, E_i, F, H of replica r, laid out alone on engine e and evaluated, into
// the caller's buffers (host, or device memory when ex->device_ptrs)
static int eval_outputs(Engine *e, Replica &r, sl_precision prec, double *energy, double *energy_atom,
                        double *force, double *field, const sl_exec *ex) {
    int rc = SL_OK;
    const int64_t n = r.n;
    const bool dev = ex && ex->device_ptrs;
    std::vector<double> Fh, Hh, Eh;
    double *F = force, *H = field;
    if (dev) {
        if (force) { Fh.resize(3 * n); F = Fh.data(); }
        if (field) { Hh.resize(3 * n); H = Hh.data(); }
    }
    if ((rc = e->download_ff(&r, F, H))) return rc;
    if ((rc = e->ensure_obs(1))) return rc;
    const Sys S = e->sys();
    if (prec == SL_FP64) launch_observe(S, e->w64, e->chunks, e->n_chunks, e->chunk_ptr, e->partial, e->obs, e->st);
    else launch_observe(S, e->w32, e->chunks, e->n_chunks, e->chunk_ptr, e->partial, e->obs, e->st);
    double ob[NOBS];
    HIPCHK(hipMemcpyAsync(ob, e->obs, sizeof(ob), hipMemcpyDeviceToHost, e->st));
    HIPCHK(hipStreamSynchronize(e->st));
    double *Ea = energy_atom;
    if (dev && energy_atom) { Eh.resize(n); Ea = Eh.data(); }
    if (Ea) {
        if (prec == SL_FP64) rc = e->download_rows(&r, e->w64.Ei, 1, 1, Ea);
        else rc = e->download_rows(&r, e->w32.Ei, 1, 1, Ea);
        if (rc) return rc;
    }
    const double Etot = ob[0] + ob[2];
    hipStream_t ust = ex && ex->hip_stream ? (hipStream_t)ex->hip_stream : e->st;
    if (dev) {
        if (energy) HIPCHK(hipMemcpyAsync(energy, &Etot, 8, hipMemcpyHostToDevice, ust));
        if (force) HIPCHK(hipMemcpyAsync(force, Fh.data(), 24 * n, hipMemcpyHostToDevice, ust));
        if (field) HIPCHK(hipMemcpyAsync(field, Hh.data(), 24 * n, hipMemcpyHostToDevice, ust));
        if (energy_atom) HIPCHK(hipMemcpyAsync(energy_atom, Eh.data(), 8 * n, hipMemcpyHostToDevice, ust));
        HIPCHK(hipStreamSynchronize(ust));
    } else if (energy) {
        *energy = Etot;
    }
    if (ob[NOBS - 1] != 0) return fail(SL_E_NONFINITE, "non-finite energy, force or state");
    return SL_OK;
}

extern "C" int nep_spin_eval(const nep_model *m, const sl_system_view *sys, sl_precision prec, double *energy,
                             double *energy_atom, double *force, double *field, const sl_exec *ex) {
    if (!m) return fail(SL_E_INVALID, "model is NULL");
    std::lock_guard<std::mutex> lk(const_cast<nep_model *>(m)->eval_mu);
    if (sys && sys->n_atoms == 0) return eval_empty(prec, energy, ex);
    Replica r;
    Engine *e = nullptr;
    int rc = eval_common(m, sys, prec, r, e);
    if (rc) return rc;
    return eval_outputs(e, r, prec, energy, energy_atom, force, field, ex);
}

extern "C" int nep_spin_eval_noalloc(const nep_model *m, const sl_system_view *sys, sl_precision prec,
                                     double *energy, double *energy_atom, double *force, double *field,
                                     const sl_exec *ex) {
    if (!m) return fail(SL_E_INVALID, "model is NULL");
    int rc = check_prec(prec);
    if (rc) return rc;
    // every call in this process shares the current GPU's scratch array
    static std::mutex scratch_mu;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (sys && sys->n_atoms == 0) return eval_empty(prec, energy, ex);
    void *base = nullptr;
    size_t bytes = 0;
    if (scratch_area(&base, &bytes) != 0)
        return fail(SL_E_DEVICE, "no device, or the static scratch area could not be resolved");
    Replica r;
    if ((rc = make_replica(sys, nullptr, nullptr, nullptr, false, r, m->structural))) return rc;
    Engine e;
    e.arena = static_cast<char *>(base);
    e.arena_cap = bytes;
    e.M = const_cast<nep_model *>(m);
    e.prec = prec;
    e.st = ex && ex->hip_stream ? (hipStream_t)ex->hip_stream : nullptr;
    if ((rc = e.set_layout({&r}))) return rc;
    if ((rc = e.check_flags())) return rc;
    return eval_outputs(&e, r, prec, energy, energy_atom, force, field, ex);
}

extern "C" int nep_spin_descriptors(const nep_model *m, const sl_system_view *sys, sl_precision prec, double *q,
                                    double *Fp, const sl_exec *ex) {
    if (!m) return fail(SL_E_INVALID, "model is NULL");
    std::lock_guard<std::mutex> lk(const_cast<nep_model *>(m)->eval_mu);
    if (sys && sys->n_atoms == 0) return check_prec(prec);
    Replica r;
    Engine *e = nullptr;
    int rc = eval_common(m, sys, prec, r, e);
    if (rc) return rc;
    const bool dev = ex && ex->device_ptrs;
    const int nd = m->structural ? DS : ND;   // row width the caller receives
    std::vector<double> qh, fh;
    double *Q = q, *P = Fp;
    if (dev) {
        if (q) { qh.resize((size_t)r.n * nd); Q = qh.data(); }
        if (Fp) { fh.resize((size_t)r.n * nd); P = fh.data(); }
    }
    if (Q) rc = prec == SL_FP64 ? e->download_rows(&r, e->w64.q, nd, DP, Q) : e->download_rows(&r, e->w32.q, nd, DP, Q);
    if (rc) return rc;
    if (P) rc = prec == SL_FP64 ? e->download_rows(&r, e->w64.Fp, nd, DP, P) : e->download_rows(&r, e->w32.Fp, nd, DP, P);
    if (rc) return rc;
    if (dev) {
        hipStream_t ust = ex->hip_stream ? (hipStream_t)ex->hip_stream : e->st;
        if (q) HIPCHK(hipMemcpyAsync(q, qh.data(), qh.size() * 8, hipMemcpyHostToDevice, ust));
        if (Fp) HIPCHK(hipMemcpyAsync(Fp, fh.data(), fh.size() * 8, hipMemcpyHostToDevice, ust));
        HIPCHK(hipStreamSynchronize(ust));
    }
    return SL_OK;
}

// ---------------------------------------------------------------------------
// single-system simulation
// ---------------------------------------------------------------------------

struct sl_sim {
    Engine eng;
    Replica r;
};

static void fill_obs(const double *o, double nfe, int64_t step, int64_t n_atoms, sl_observables *out, int passes,
                     double change) {
    out->step = step;
    out->spin_passes = passes;
    out->spin_change = change;
    out->E_pot = o[0];
    out->E_kin = o[1];
    out->E_zeeman = o[2];
    out->T_lattice = n_atoms ? 2.0 * o[1] / (3.0 * n_atoms * KB) : 0.0;
    out->T_spin = o[4] != 0 ? o[3] / (2.0 * KB * o[4]) : 0.0;
    for (int a = 0; a < 3; a++) out->M[a] = nfe > 0 ? o[5 + a] / nfe : 0.0;
    out->spin_length = nfe > 0 ? o[8] / nfe : 0.0;
    out->mid_capped = (int32_t)o[9];
}

extern "C" int sl_create(const nep_model *m, const sl_system_view *sys, const double *vel, const int32_t *colour,
                         const sl_integrator_params *ip, sl_precision prec, sl_sim **out) {
    if (!out) return fail(SL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!m || !ip) return fail(SL_E_INVALID, "model and integrator parameters are required");
    int rc = check_prec(prec);
    if (rc) return rc;
    auto s = std::make_unique<sl_sim>();
    if ((rc = make_replica(sys, vel, colour, ip, !m->structural, s->r, m->structural))) return rc;
    s->eng.M = const_cast<nep_model *>(m);
    s->eng.prec = prec;
    s->eng.K_corr = ip->K_corr;
    s->eng.sc_tol = ip->sc_tol;
    s->eng.sc_max = ip->sc_max;
    s->eng.sc_depth = ip->sc_tol > 0 ? ip->sc_depth : 0;
    s->eng.sc_reg = ip->sc_reg;
    if ((rc = s->eng.set_layout({&s->r}))) return rc;
    std::vector<int> bad;
    if ((rc = settle_layout(s->eng, bad))) return rc;
    if (bad[0] == SL_E_INVALID) return fail(SL_E_INVALID, colour_msg);
    if (bad[0]) return fail(bad[0], "neighbour list capacity exceeded");
    *out = s.release();
    return SL_OK;
}

extern "C" int sl_integrate_steps(sl_sim *s, int64_t n_steps, sl_observables *per_step_out) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    if (n_steps < 0) return fail(SL_E_INVALID, "n_steps must be non-negative");
    Engine &e = s->eng;
    // steps are queued in chunks; a replica paused for recolouring inside a
    // chunk idles through the rest of it, so chunks stay short
    const int64_t chunk = 16;
    std::vector<double> h(chunk * NOBS);
    std::vector<RepDev> d;
    int rc;
    if ((rc = e.ensure_obs(chunk))) return rc;
    if ((rc = e.read_reps(d))) return rc;
    int64_t step = d[0].step;
    int64_t done = 0;
    while (done < n_steps) {
        const int64_t k = std::min(chunk, n_steps - done);
        e.log_passes.clear();
        e.log_change.clear();
        for (int64_t q = 0; q < k; q++) e.step(e.obs + q * NOBS);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h.data(), e.obs, k * NOBS * 8, hipMemcpyDeviceToHost, e.st));
        HIPCHK(hipStreamSynchronize(e.st));
        e.prof_collect();
        if ((rc = e.check_flags())) return rc;
        if ((rc = e.read_reps(d))) return rc;
        const int64_t ran = d[0].step - step;       // steps completed in this chunk
        for (int64_t q = 0; q < ran; q++) {
            const double *o = h.data() + q * NOBS;
            const bool sc = e.sc_tol > 0 && q < (int64_t)e.log_passes.size();
            if (per_step_out)
                fill_obs(o, (double)s->r.n_fe, step + q + 1, s->r.n, per_step_out + done + q,
                         sc ? e.log_passes[q] : e.K_corr + 1, sc ? e.log_change[q] : 0.0);
            if (o[NOBS - 1] != 0) return fail(SL_E_NONFINITE, "state became non-finite at step " + std::to_string(step + q + 1));
        }
        done += ran;
        step += ran;
        if (d[0].failed & 1) return fail(SL_E_OVERFLOW, "neighbour list capacity exceeded");
        if (d[0].failed & 2) return fail(SL_E_INVALID, colour_msg);
        if (d[0].failed & 4) {
            // a same-colour pair entered the list shell: new colouring, then go on
            if ((rc = recolour_replica(e, &s->r))) return rc;
            if ((rc = e.set_layout({&s->r}))) return rc;
            std::vector<int> bad;
            if ((rc = settle_layout(e, bad))) return rc;
            if (bad[0]) return fail(bad[0], bad[0] == SL_E_INVALID ? colour_msg : "neighbour list capacity exceeded");
        } else if (ran < k) {
            return fail(SL_E_DEVICE, "replica stopped before its steps were done");
        }
    }
    return SL_OK;
}

extern "C" int sl_get_colour(const sl_sim *s, int32_t *colour, int64_t *n_recolour) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    const Replica &r = s->r;
    if (colour) {
        for (int64_t q = 0; q < r.n; q++) colour[q] = -1;
        for (int64_t q = 0; q < r.n_fe; q++) colour[r.fe_idx[q]] = r.colour_fe[q];
    }
    if (n_recolour) *n_recolour = r.n_recolour;
    return SL_OK;
}

extern "C" int sl_get_state(const sl_sim *s, double *pos, double *vel, double *spin, int64_t *step) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    sl_sim *x = const_cast<sl_sim *>(s);
    int rc = x->eng.download(&x->r, pos, vel, spin);
    if (rc) return rc;
    if (step) {
        RepDev d;
        HIPCHK(hipMemcpy(&d, x->eng.rep, sizeof(RepDev), hipMemcpyDeviceToHost));
        *step = d.step;
    }
    return SL_OK;
}

extern "C" int sl_set_state(sl_sim *s, const double *pos, const double *vel, const double *spin, int64_t step) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    if (!pos || !vel || !spin) return fail(SL_E_INVALID, "pos, vel and spin are required");
    Replica &r = s->r;
    RepDev d;
    HIPCHK(hipMemcpy(&d, s->eng.rep, sizeof(RepDev), hipMemcpyDeviceToHost));
    r.dev = d;
    r.dev.step = step;
    r.dev.active = 1;
    r.pos.assign(pos, pos + 3 * r.n);
    r.vel.assign(vel, vel + 3 * r.n);
    r.spin.assign(spin, spin + 3 * r.n);
    for (int64_t q = 0; q < r.n - r.n_fe; q++) {
        const int c = r.ge_idx[q];
        r.spin[3 * c] = r.spin[3 * c + 1] = r.spin[3 * c + 2] = 0;
    }
    r.fe_off = r.ge_off = -1;   // re-upload from the host copies
    s->eng.reps.clear();
    int rc = s->eng.set_layout({&r});
    if (rc) return rc;
    std::vector<int> bad;
    if ((rc = settle_layout(s->eng, bad))) return rc;
    if (bad[0]) return fail(bad[0], bad[0] == SL_E_INVALID ? colour_msg : "neighbour list capacity exceeded");
    return SL_OK;
}

extern "C" int sl_profile_enable(sl_sim *s, unsigned mask) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    s->eng.prof_mask = mask & ((1u << SL_NPROF) - 1);
    return SL_OK;
}

extern "C" int sl_profile_read(sl_sim *s, double *ms_total, int64_t *launches) {
    if (!s) return fail(SL_E_INVALID, "sim is NULL");
    for (int g = 0; g < SL_NPROF; g++) {
        if (ms_total) ms_total[g] = s->eng.prof_ms[g];
        if (launches) launches[g] = s->eng.prof_n[g];
        s->eng.prof_ms[g] = 0;
        s->eng.prof_n[g] = 0;
    }
    return SL_OK;
}

extern "C" int sl_destroy(sl_sim *s) {
    delete s;
    return SL_OK;
}

// ---------------------------------------------------------------------------
// replica server
// ---------------------------------------------------------------------------

struct sl_server {
    nep_model *m = nullptr;
    sl_server_config cfg{};
    Engine eng;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Replica *> queue;
    std::map<uint64_t, std::unique_ptr<Replica>> all;
    std::vector<Replica *> resident;
    std::thread worker;
    bool stop = false;
    int worker_error = 0;
    std::string worker_msg;
    uint64_t next_id = 1;
    double t0 = 0;
    size_t budget = 0, used = 0;
    int64_t batched_steps = 0;
    double atom_steps = 0, busy = 0;
    // host time between batches: re-layouts (count, seconds) and all gaps
    int64_t relayouts = 0;
    double relayout_s = 0, gap_s = 0;
    size_t pending = 0;

    void run();
};

static double pct(std::vector<double> v, double p) {
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    const double x = p * (v.size() - 1);
    const size_t a = (size_t)x;
    const size_t b = std::min(a + 1, v.size() - 1);
    return v[a] + (v[b] - v[a]) * (x - a);
}

void sl_server::run() {
    const int spb = std::max(1, cfg.steps_per_batch);
    std::vector<hipEvent_t> ev(spb + 1);
    for (auto &e : ev) (void)hipEventCreate(&e);
    std::vector<double> hobs;
    double last_done_t = 0;
    for (;;) {
        std::vector<Replica *> next;
        bool changed = false;
        {
            std::unique_lock<std::mutex> lk(mu);
            // retire finished or failed replicas
            std::vector<Replica *> keep;
            for (Replica *r : resident) {
                if (r->steps_done >= r->n_steps || r->state == SL_FAILED) {
                    lk.unlock();
                    r->pos.assign(3 * r->n, 0);
                    r->vel.assign(3 * r->n, 0);
                    r->spin.assign(3 * r->n, 0);
                    int rc = eng.download(r, r->pos.data(), r->vel.data(), r->spin.data());
                    lk.lock();
                    if (rc && r->state != SL_FAILED) {
                        r->state = SL_FAILED;
                        r->error = rc;
                    }
                    if (r->state != SL_FAILED) r->state = SL_DONE;
                    r->t_done = now_s() - t0;
                    used -= r->bytes;
                    pending--;
                    changed = true;
                } else {
                    keep.push_back(r);
                }
            }
            // admit queued replicas while slots and budget allow (in arrival order)
            while (!queue.empty() && (int)keep.size() < cfg.max_slots && used + queue.front()->bytes <= budget) {
                Replica *r = queue.front();
                queue.pop_front();
                r->state = SL_RUNNING;
                r->t_admit = now_s() - t0;
                used += r->bytes;
                keep.push_back(r);
                changed = true;
            }
            if (changed) done_cv.notify_all();
            if (keep.empty() && queue.empty()) {
                resident.clear();
                if (stop) break;
                cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop && queue.empty()) break;
                continue;
            }
            next = keep;
        }
        // replicas paused on a colour conflict get a new colouring first
        int rc = SL_OK;
        for (Replica *r : next)
            if (r->need_recolour && r->slot >= 0 && !rc) {
                rc = recolour_replica(eng, r);
                r->need_recolour = false;
                changed = true;
            }
        if (!rc && (changed || next != eng.reps)) {
            const double tl = now_s();
            rc = eng.set_layout(next);
            std::vector<int> bad;
            if (!rc) rc = settle_layout(eng, bad, false);
            std::lock_guard<std::mutex> lk(mu);
            relayouts++;
            relayout_s += now_s() - tl;
            resident = next;
            for (size_t a = 0; a < bad.size() && !rc; a++)
                if (bad[a] && next[a]->state == SL_RUNNING) {
                    next[a]->state = SL_FAILED;
                    next[a]->error = bad[a];
                }
        }
        if (rc) {
            std::lock_guard<std::mutex> lk(mu);
            resident = next;
            for (Replica *r : next) {
                r->state = SL_FAILED;
                r->error = rc;
            }
            worker_error = rc;
            worker_msg = g_err;
            continue;
        }
        // batched steps of every resident replica
        int64_t k = spb;
        for (Replica *r : next) k = std::min<int64_t>(k, r->n_steps - r->steps_done);
        if (k <= 0) k = 1;
        if (eng.ensure_obs(k)) {
            std::lock_guard<std::mutex> lk(mu);
            worker_error = SL_E_OOM;
            for (Replica *r : next) { r->state = SL_FAILED; r->error = SL_E_OOM; }
            continue;
        }
        const double tb = now_s();
        (void)hipEventRecord(ev[0], eng.st);
        const size_t nr = next.size();
        for (int64_t q = 0; q < k; q++) {
            eng.step(eng.obs + q * nr * NOBS);
            (void)hipEventRecord(ev[q + 1], eng.st);
        }
        hobs.resize(k * nr * NOBS);
        (void)hipMemcpyAsync(hobs.data(), eng.obs, hobs.size() * 8, hipMemcpyDeviceToHost, eng.st);
        hipError_t herr = hipStreamSynchronize(eng.st);
        std::vector<RepDev> dv;
        int frc = herr == hipSuccess ? SL_OK : SL_E_DEVICE;
        if (!frc) frc = eng.read_reps(dv);
        const double te = now_s();
        std::vector<double> lat(k);
        for (int64_t q = 0; q < k; q++) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[q], ev[q + 1]);
            lat[q] = ms * 1e-3;
        }
        // the first step of a batch also waited for the host
        const double gap = last_done_t > 0 ? std::max(0.0, tb - last_done_t) : 0.0;
        lat[0] += gap;
        last_done_t = te;
        {
            std::lock_guard<std::mutex> lk(mu);
            batched_steps += k;
            busy += te - tb;
            gap_s += gap;
            for (size_t a = 0; a < nr; a++) {
                Replica *r = next[a];
                if (r->state != SL_RUNNING) continue;
                if (frc) {
                    r->state = SL_FAILED;
                    r->error = frc;
                    continue;
                }
                // steps this replica completed in the batch (it stops early on a
                // failure or a colour conflict)
                const int64_t kk = std::max<int64_t>(
                    0, std::min<int64_t>(dv[a].step - (r->step0 + r->steps_done), r->n_steps - r->steps_done));
                for (int64_t q = 0; q < kk; q++) {
                    const double *o = hobs.data() + (q * nr + a) * NOBS;
                    if (o[NOBS - 1] != 0 && r->state == SL_RUNNING) {
                        r->state = SL_FAILED;
                        r->error = SL_E_NONFINITE;
                    }
                    r->lat.push_back(lat[q]);
                }
                if (r->state == SL_RUNNING && (dv[a].failed & 3)) {
                    r->state = SL_FAILED;
                    r->error = (dv[a].failed & 1) ? SL_E_OVERFLOW : SL_E_INVALID;
                }
                if (r->state == SL_RUNNING && (dv[a].failed & 4)) r->need_recolour = true;
                if (kk > 0) {
                    std::memcpy(r->obs_last, hobs.data() + ((kk - 1) * nr + a) * NOBS, NOBS * 8);
                    r->obs_step = r->step0 + r->steps_done + kk;
                    r->last_passes = dv[a].sc_passes;
                    r->last_change = dv[a].sc_last;
                }
                r->steps_done += kk;
                atom_steps += (double)kk * r->n;
            }
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
}

extern "C" int sl_server_create(const nep_model *m, const sl_server_config *cfg, sl_server **out) {
    if (!out) return fail(SL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!m || !cfg) return fail(SL_E_INVALID, "model and config are required");
    int rc = check_prec(cfg->precision);
    if (rc) return rc;
    if (cfg->max_slots < 1 || cfg->steps_per_batch < 1 || cfg->K_corr < 0 || cfg->K_corr > 64)
        return fail(SL_E_INVALID, "max_slots and steps_per_batch must be >= 1, K_corr in [0, 64]");
    auto s = std::make_unique<sl_server>();
    s->m = const_cast<nep_model *>(m);
    s->cfg = *cfg;
    s->eng.M = s->m;
    s->eng.prec = cfg->precision;
    s->eng.K_corr = cfg->K_corr;
    size_t budget = cfg->hbm_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        const size_t reserve = (size_t)4 << 30;
        budget = fr > reserve ? fr - reserve : fr / 2;
    }
    s->budget = budget;
    s->t0 = now_s();
    sl_server *raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    *out = s.release();
    return SL_OK;
}

extern "C" int sl_replica_submit(sl_server *sv, const sl_system_view *sys, const double *vel, const int32_t *colour,
                                 const sl_integrator_params *ip, int64_t n_steps, uint64_t *id_out) {
    if (!sv || !ip || !id_out) return fail(SL_E_INVALID, "server, params and id_out are required");
    if (ip->K_corr != sv->cfg.K_corr) return fail(SL_E_INVALID, "K_corr must equal the server's");
    if (ip->sc_tol != 0 && ip->sc_depth != 0)
        return fail(SL_E_INVALID, "replicas in the server iterate the midpoint without mixing: sc_depth must be 0");
    if (n_steps < 1) return fail(SL_E_INVALID, "n_steps must be >= 1");
    auto r = std::make_unique<Replica>();
    int rc = make_replica(sys, vel, colour, ip, !sv->m->structural, *r, sv->m->structural);
    if (rc) return rc;
    r->n_steps = n_steps;
    r->bytes = sl_replica_bytes(r->n, sv->cfg.precision);
    if (r->bytes > sv->budget) return fail(SL_E_OOM, "replica larger than the whole HBM budget");
    r->step0 = r->dev.step;
    r->dev.step_end = r->dev.step + n_steps;
    std::lock_guard<std::mutex> lk(sv->mu);
    r->id = sv->next_id++;
    r->t_submit = now_s() - sv->t0;
    r->state = SL_QUEUED;
    *id_out = r->id;
    sv->queue.push_back(r.get());
    sv->all[r->id] = std::move(r);
    sv->pending++;
    sv->cv.notify_all();
    return SL_OK;
}

extern "C" int sl_replica_poll(sl_server *sv, uint64_t id, sl_replica_status *out) {
    if (!sv || !out) return fail(SL_E_INVALID, "server and out are required");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(SL_E_NOTFOUND, "unknown replica id");
    Replica *r = it->second.get();
    out->state = r->state;
    out->error = r->error;
    out->steps_done = r->steps_done;
    out->n_steps = r->n_steps;
    out->t_submit = r->t_submit;
    out->t_admit = r->t_admit;
    out->t_done = r->t_done;
    out->step_latency_p50 = pct(r->lat, 0.50);
    out->step_latency_p99 = pct(r->lat, 0.99);
    out->n_latency_samples = (int64_t)r->lat.size();
    return SL_OK;
}

extern "C" int sl_replica_fetch(sl_server *sv, uint64_t id, double *pos, double *vel, double *spin,
                                sl_observables *obs) {
    if (!sv) return fail(SL_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(SL_E_NOTFOUND, "unknown replica id");
    Replica *r = it->second.get();
    if (r->state == SL_QUEUED || r->state == SL_RUNNING) return fail(SL_E_BUSY, "replica not finished");
    if (r->state == SL_FAILED) return fail(r->error ? r->error : SL_E_NONFINITE, "replica failed");
    if (pos) std::memcpy(pos, r->pos.data(), 24 * r->n);
    if (vel) std::memcpy(vel, r->vel.data(), 24 * r->n);
    if (spin) std::memcpy(spin, r->spin.data(), 24 * r->n);
    if (obs) {
        const bool sc = r->dev.sc_tol > 0;
        fill_obs(r->obs_last, (double)r->n_fe, r->obs_step, r->n, obs, sc ? r->last_passes : sv->eng.K_corr + 1,
                 sc ? r->last_change : 0.0);
    }
    return SL_OK;
}

extern "C" int sl_server_drain(sl_server *sv) {
    if (!sv) return fail(SL_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->done_cv.wait(lk, [&] { return sv->pending == 0 || sv->worker_error != 0; });
    if (sv->worker_error) return fail(sv->worker_error, "server worker: " + sv->worker_msg);
    return SL_OK;
}

extern "C" int sl_server_stats(sl_server *sv, int64_t *batched_steps, double *atom_steps, double *busy_s) {
    if (!sv) return fail(SL_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (batched_steps) *batched_steps = sv->batched_steps;
    if (atom_steps) *atom_steps = sv->atom_steps;
    if (busy_s) *busy_s = sv->busy;
    return SL_OK;
}

extern "C" int sl_server_host_stats(sl_server *sv, int64_t *relayouts, double *relayout_s, double *gap_s) {
    if (!sv) return fail(SL_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (relayouts) *relayouts = sv->relayouts;
    if (relayout_s) *relayout_s = sv->relayout_s;
    if (gap_s) *gap_s = sv->gap_s;
    return SL_OK;
}

extern "C" int sl_server_destroy(sl_server *sv) {
    if (!sv) return SL_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    delete sv;
    return SL_OK;
}
