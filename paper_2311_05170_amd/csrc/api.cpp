// C-ABI layer: context lifetime, device buffers, and the per-step launch
// sequences of Algorithm 3 (Step 1 on T_H, Steps 3-4 on the subdomains).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "lp_internal.h"

namespace {

thread_local std::string g_err;

lp_status fail(lp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            return fail(LP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));     \
    } while (0)

}  // namespace

lp_status lp::set_error(lp_status s, const std::string &msg) { return fail(s, msg); }

// Scratch of lp_local_step_noalloc: one array per device, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, taken once per device at lp_setup
// with that device current, and only that address is handed to kernels.
#define LP_NOALLOC_SCRATCH_BYTES (8LL << 20)
static __device__ __align__(256) unsigned char scratch[LP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device (first call per device)
lp_status init_static_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return fail(LP_ERR_DEVICE, "device id out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return LP_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (unsigned char *)ptr;
    return LP_OK;
}

lp_status static_scratch(int device, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES || !g_scratch_ptr[device])
        return fail(LP_ERR_STATE, "static scratch of this device was not set up (lp_setup on it first)");
    *out = g_scratch_ptr[device];
    return LP_OK;
}

}  // namespace

struct lp_ctx {
    lp::Plan P;
    lp::Coef co{};
    lp::RefData ref{};
    lp_params prm{};
    std::vector<lp_params> samples_h;  // every sample's parameters, as given to lp_setup
    lp_options opt{};
    lp_allocator alloc{};
    bool has_alloc = false;
    std::vector<void *> owned;
    int64_t n = 0;                 // completed local steps
    bool coarse_pending = false;
    bool one_grid = false;             // Algorithm 1: the coarse step is the whole step
    bool lag_merged = false;           // lagged e^n from the merged correction (LP_LAG_MERGED)
    // Parameter samples advanced together (lp_options.nsamples): every system
    // list holds the systems of sample 0, then of sample 1, ...; the fields
    // read by position on a lattice (coarse states, prolongations, loads,
    // merged output, Newton iterates) live in one arena block per sample,
    // zs doubles apart (SysDesc::zo = sample * zs).
    int ns = 1;
    int np1 = 0, no1 = 0;              // porous / conduit subdomains per sample
    long long zs = 0;
    double *arena = nullptr;
    // Coarse states live in a ring of RING slots (time m in slot m % RING).
    // The coarse step runs on an internal stream: it never reads local
    // results, so coarse steps run ahead of the local stage (up to RING - 2
    // steps).  A slot is rewritten only after the local step that last reads
    // it has finished.
    static constexpr int RING = 8;
    static constexpr int FSLOTS = 8;   // factor slots of the local Oseen operators (<= RING, a divisor of it)
    hipStream_t cstream = nullptr;
    hipEvent_t ev_coarse[RING] = {}, ev_local[RING] = {};
    hipEvent_t ev_cpor[RING] = {};     // coarse porous solves of a level done (they run on a factor stream)
    hipEvent_t ev_pro[RING] = {};      // prolongation slot of a level written (on its factor stream)
    // the local porous batch of step m runs on factor stream m % 2 (mixed
    // path), after that step's Oseen factorisation, beside the Oseen solves, or
    // on the caller's stream ahead of them (FP64 path); four streams in all,
    // within HIP's default of four hardware queues per process
    hipEvent_t ev_por = nullptr;                       // porous batch of the latest local step done
    // The local Oseen operator of step m depends only on u_cH^m, so its
    // assembly and factorisation run on factor stream m % 2 as soon as coarse
    // step m is done, overlapping the solves of step m-1 and the factorisation
    // of step m-1 (one workgroup per system leaves most CUs to the other).
    // The band of step m uses slot m % 2 (ordered by the stream), its
    // prolonged fields ring slot m % RING, its factors slot m % FSLOTS,
    // rewritten once local step m - FSLOTS has finished.
    hipStream_t fstream[2] = {};
    hipEvent_t ev_fac[FSLOTS] = {};
    // Graph mode (lp_options.graphs): each launch sequence that one stream
    // runs between event operations (the coarse porous and Navier-Stokes
    // parts, the prolongation, the assembly and factorisation, the porous
    // batch, the local Oseen right-hand sides, refinement and merge) is
    // captured once per (sequence, ring slot) on lstream, a stream that only
    // records, and replayed as a HIP graph on the stream the sequence belongs
    // to.
    static constexpr int GSLOTS = RING;
    bool graphs = false;
    hipStream_t lstream = nullptr;
    std::map<int, hipGraphExec_t> gx;
    int64_t seg_m = 0;             // the step whose launches seg() is issuing
    int key_off = 0;               // graph key offset of the local step's scratch (allocation-free variant)
    // time factors (cos t, sin t, cos^2 t) of each ring slot's level, and the
    // slot's level counter (next level of the slot, advanced by RING)
    double *tf_dev = nullptr;
    long long *level_dev = nullptr;
    double *tf_slot(int slot) const { return tf_dev + 4 * slot; }
    int64_t graph_launches = 0, graph_instantiations = 0;
    int ecur = 0;                  // correction buffers holding e^n
    bool serial = false;           // diagnostic (LP_SERIAL=1): all stages on one stream, no overlap
    bool mixed = false;

    // sizes
    long long nf2 = 0, nf1 = 0, nc2 = 0, nc1 = 0;

    // tables and descriptors
    lp::SysDesc *d_por = nullptr, *d_ose = nullptr, *d_cpor = nullptr, *d_cns = nullptr;
    int8_t *d_cls2 = nullptr, *d_cls1 = nullptr;
    int32_t *d_dof2 = nullptr, *d_dof1 = nullptr;
    lp::BandSys *d_lu_por = nullptr, *d_lu_ose = nullptr, *d_lu_cpor = nullptr, *d_lu_cns = nullptr;
    lp::BandSys *d_sv_por = nullptr, *d_sv_ose = nullptr, *d_sv_cpor = nullptr, *d_sv_cns = nullptr;
    int32_t *d_own[2][2][4] = {};  // [region][axis][own2_lo, own2_n, own1_lo, own1_n]

    // manufactured data on both grids
    double *ex_f[6] = {}, *ex_c[6] = {};
    double *ld_f[5][3] = {}, *ld_c[5][3] = {};

    // coarse states (two time levels)
    double *cP[RING] = {}, *cU[RING] = {}, *cp[RING] = {};
    double *nwt_e = nullptr, *nwt_e1 = nullptr;
    int *d_done = nullptr, *d_its = nullptr, *d_flags = nullptr;
    // factorisation monitor, run-long maxima (float bits): growth and
    // inverse smallest relative pivot of the local systems, then the coarse ones
    float *d_lustat = nullptr;
    lp::Coef *d_co = nullptr;          // the coefficients every assembly and residual kernel reads
    // run-long refinement totals (largest sweep count, largest final relative
    // residual as double bits), folded in by the local finalize kernels
    int *d_irmax = nullptr;
    unsigned long long *d_irrel = nullptr;

    // prolonged coarse fields on the fine lattices.  Setup: the porous
    // pressures and the velocity of level 0, for the initial corrections.
    // Per step, slot m % RING (written after coarse step m, on its stream):
    // u^m (2 fields), u^(m-1) (2 fields), p_F^(m-1) on P2, then p^m on P1.
    double *pro_P1 = nullptr, *pro_U1 = nullptr;
    double *pro_ring = nullptr;
    long long pro_stride = 0;
    double *pro_slot(int s) const { return pro_ring + (long long)s * pro_stride; }

    // local corrections (two time levels) and merged output
    double *e2[2] = {}, *e1[2] = {};
    double *m_P = nullptr, *m_U = nullptr, *m_p = nullptr;

    // linear algebra storage
    void *band_por = nullptr, *band_ose[2] = {};          // float (mixed) or double
    double *band_cpor = nullptr, *band_cns = nullptr;
    // explicit inverses of the small coarse matrices (column-major), the
    // identity right-hand sides that produce them, and their solve lists
    double *inv_cp = nullptr, *inv_cn = nullptr, *eye_cp = nullptr, *eye_cn = nullptr;
    lp::BandSys *d_iv_cpor = nullptr, *d_iv_cns = nullptr;
    void *fac_por = nullptr, *fac_ose[FSLOTS] = {};       // factors (layout: fac_layout)
    double *pro_Pb[2] = {};                              // the porous batch's prolonged inputs, per step parity:
                                                         // p^(n+1) (3 fields), p^n (3 fields), u_y^n
    double *fac_cpor = nullptr, *fac_cns = nullptr;
    double *b_por = nullptr, *x_por = nullptr, *r_por = nullptr;
    double *b_ose = nullptr, *x_ose = nullptr, *r_ose = nullptr;
    double *b_cp = nullptr, *x_cp = nullptr, *r_cp = nullptr;
    double *b_cn = nullptr, *x_cn = nullptr, *r_cn = nullptr;
    int *conv_por = nullptr, *conv_ose = nullptr, *conv_cp = nullptr, *conv_cn = nullptr;
    double *rel_por = nullptr, *rel_ose = nullptr, *rel_cp = nullptr, *rel_cn = nullptr;
    int *sw_por = nullptr, *sw_ose = nullptr, *sw_cp = nullptr, *sw_cn = nullptr;

    int maxbw_por = 0, maxbw_ose = 0, maxn_por = 0, maxn_ose = 0;
    // Krylov path of the local Oseen systems (boxes too wide for the band
    // factorisation, or LP_KRYLOV): FGMRES(m) preconditioned by restricted
    // additive Schwarz over strips whose Stokes-part band matrices are
    // factored once at setup
    bool krylov = false;
    bool have_dense = false, have_strips = false;  // resources of each local Oseen path
    int gm_m = 0;
    int krylov_cycles() const { return opt.krylov_cycles > 0 ? opt.krylov_cycles : opt.max_ir; }
    int gm_reorth = 0;             // second Gram-Schmidt pass in the Arnoldi steps (LP_GM_REORTH)
    // setup-time autotuning (lp_options.autotune): measured milliseconds of
    // one local Oseen solve batch by each path, and what was chosen
    bool tuned = false;
    double tune_dense_ms = 0.0, tune_krylov_ms = 0.0;
    lp::SysDesc *d_strip = nullptr;
    int32_t *d_strip_parent = nullptr, *d_smap = nullptr;
    int8_t *d_sown = nullptr;
    lp::BandSys *d_lu_strip = nullptr, *d_sv_strip = nullptr;
    void *band_strip = nullptr, *fac_strip = nullptr;
    int maxbw_strip = 0, maxn_strip = 0;
    double *gm_V = nullptr, *gm_Z = nullptr, *gm_H = nullptr, *gm_cs = nullptr, *gm_sn = nullptr, *gm_g = nullptr;
    double *gm_bn = nullptr, *gm_w = nullptr, *s_rs = nullptr, *s_zs = nullptr;
    int *gm_done = nullptr, *gm_kd = nullptr, *gm_tot = nullptr, *s_done = nullptr;
    // largest local P2 lattice per batch (node blocks of the gather kernels)
    int nodes_por = 0, nodes_ose = 0, nodes_cpor = 0, nodes_cns = 0;
    int tiles_ose = 0, tiles_por = 0;  // most residual tiles of a local Oseen / porous box
    // local Oseen assembly into bands cleared once at setup, each entry's
    // first element storing instead of adding (LP_OSEEN_ASM=0: cleared and
    // read back every step)
    bool asm_first_write = true;
    int rblk_ose = 0, rblk_por = 0;    // residual blocks per box (each takes every rblk-th tile)
    // residual norm partials and arrival counters, one set per batch (the
    // batches run on different streams)
    double *part_por = nullptr, *part_ose = nullptr, *part_cp = nullptr, *part_cn = nullptr;
    int *tick_por = nullptr, *tick_ose = nullptr, *tick_cp = nullptr, *tick_cn = nullptr;
    int *tick_dn = nullptr, *tick_dp = nullptr;        // last-block tickets of the fused coarse kernels
    long long scratch_part_por = 0, scratch_part_ose = 0;   // doubles of norm partials per batch
    int device = 0;                    // HIP device the context was set up on
    double *lu_dummy = nullptr;        // sink of the factorisation's masked stores
    long long lu_dummy_coarse_off = 0;
    int lu_variant = 0;                // factorisation kernel of the porous and coarse systems (0: default)
    int lu_variant_ose = 9;            // of the local Oseen systems (blocked on the matrix cores with lookahead)
    int lu_variant_cns = 9;            // of the coarse Navier-Stokes Jacobian (9: blocked on the matrix cores with lookahead)
    int solve_depth = 0;               // factor columns prefetched by the band solves (16, 32, 64 (FP32); 0 = by precision)
    // device constants read by masked loads: 512 zero doubles (a zero column
    // for the solves), then 1.0 as double, then 1.0f as float
    double *consts = nullptr;
    template <typename T>
    const T *const_one() const {
        return sizeof(T) == 8 ? (const T *)(consts + 512) : (const T *)(consts + 513);
    }

    // stage timers (HIP events on the caller's stream)
    uint32_t tmask = 0;
    struct Rec { hipEvent_t a, b; int stage; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double tms[LP_T_COUNT] = {};
    int64_t tcnt[LP_T_COUNT] = {};

    hipEvent_t event() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }

    ~lp_ctx() {
        if (cstream) (void)hipStreamSynchronize(cstream);
        for (int i = 0; i < RING; ++i) {
            if (ev_coarse[i]) (void)hipEventDestroy(ev_coarse[i]);
            if (ev_local[i]) (void)hipEventDestroy(ev_local[i]);
            if (ev_cpor[i]) (void)hipEventDestroy(ev_cpor[i]);
            if (ev_pro[i]) (void)hipEventDestroy(ev_pro[i]);
        }
        if (cstream) (void)hipStreamDestroy(cstream);
        if (serial) fstream[0] = fstream[1] = nullptr;
        for (int i = 0; i < 2; ++i)
            if (fstream[i]) { (void)hipStreamSynchronize(fstream[i]); (void)hipStreamDestroy(fstream[i]); }
        for (int i = 0; i < FSLOTS; ++i)
            if (ev_fac[i]) (void)hipEventDestroy(ev_fac[i]);
        if (ev_por) (void)hipEventDestroy(ev_por);
        if (lstream) { (void)hipStreamSynchronize(lstream); (void)hipStreamDestroy(lstream); }
        for (auto &kv : gx)
            if (kv.second) (void)hipGraphExecDestroy(kv.second);
        for (auto &r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
        for (void *p : owned) {
            if (has_alloc) alloc.free(p, alloc.user);
            else (void)hipFree(p);
        }
    }

    template <typename T>
    lp_status dalloc(T **p, long long count) {
        size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
        void *q = nullptr;
        if (has_alloc) q = alloc.alloc(bytes, alloc.user);
        else if (hipMalloc(&q, bytes) != hipSuccess) q = nullptr;
        if (!q) return fail(LP_ERR_ALLOC, "device allocation of " + std::to_string(bytes) + " bytes failed");
        owned.push_back(q);
        *p = (T *)q;
        return LP_OK;
    }

    template <typename T>
    lp_status upload(T **p, const std::vector<T> &v, hipStream_t st) {
        lp_status s = dalloc(p, (long long)v.size());
        if (s != LP_OK) return s;
        if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        return LP_OK;
    }
};

namespace {

#define TRY(expr)                        \
    do {                                 \
        lp_status _s = (expr);           \
        if (_s != LP_OK) return _s;      \
    } while (0)

// Scratch of the local step's refinement: residual-norm partials and
// last-block tickets of the porous and the Oseen batches (they run on
// different streams).  The context's own buffers, or a static device array
// (lp_local_step_noalloc).
struct LocalScratch {
    double *part_por, *part_ose;
    int *tick_por, *tick_ose;
};

// brackets the launches of one stage with events when its bit is set
struct StageTimer {
    lp_ctx *c;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    StageTimer(lp_ctx *c_, int stage_, hipStream_t st_) : c(c_), stage(stage_), st(st_) {
        if (stage >= 0 && (c->tmask >> stage) & 1u) {
            a = c->event();
            if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
        }
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = c->event();
        if (b && hipEventRecord(b, st) == hipSuccess) c->recs.push_back({a, b, stage});
    }
};

// Run the launches of `body` on stream st: directly, or (graph mode, no stage
// timers, from the third step on) as the HIP graph of `key`, captured and
// instantiated the first time the key is met and replayed after that.  A key
// names a launch sequence and a ring slot: every argument of the sequence is
// a function of the slot (buffers of the slot's level, the slot's time
// factors in device memory) and not of the step, so a replay does the next
// step of that slot exactly.  A key's replays all go to the same stream.
template <class F>
lp_status seg(lp_ctx *c, int key, hipStream_t st, F &&body) {
    if (!c->graphs || c->tmask || c->seg_m < 3) return body(st);
    hipGraphExec_t &ex = c->gx[key];
    if (!ex) {
        // recorded on the context's capture stream (the caller's stream may be
        // the null stream, which cannot capture), replayed on st
        hipStream_t cs = c->lstream;
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const lp_status s = body(cs);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (s != LP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess || !graph) return fail(LP_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        const hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            ex = nullptr;
            return fail(LP_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
        c->graph_instantiations += 1;
    }
    HIPCHK(hipGraphLaunch(ex, st));
    c->graph_launches += 1;
    return LP_OK;
}

// graph keys: launch sequence x step slot
enum { G_CPOR = 0, G_CNS = 1, G_CNS_REFRESH = 2, G_PROLONG = 3, G_FACTOR = 4, G_POROUS = 5, G_OSE_RHS = 6,
       G_OSE_SOLVE = 7, G_MERGE = 8 };
int gkey(int seq, int64_t m) { return seq * lp_ctx::GSLOTS + (int)(m % lp_ctx::GSLOTS); }
// the allocation-free local step's sequences read other scratch buffers
constexpr int G_NOALLOC = 1 << 12;

// Factor storage of a batch: per (system, matrix) n (2 ldf + 1) entries,
// ldf = 64 NR for the solve's NR registers per lane (L and U columns of ldf
// entries, then 1/U(k,k)), each block rounded up to 64 entries.
struct FacLayout {
    std::vector<long long> off;
    long long total = 0;
    int ldf = 0;
};

FacLayout fac_layout(const std::vector<lp::SysDesc> &v, int nmat, int maxbw) {
    FacLayout L;
    L.ldf = 64 * lp::solve_nr(maxbw);
    for (const auto &s : v)
        for (int f = 0; f < nmat; ++f) {
            L.off.push_back(L.total);
            L.total += ((long long)s.ndof * (2 * L.ldf + 1) + 63) / 64 * 64;
        }
    return L;
}

std::vector<lp::BandSys> lu_list(const std::vector<lp::SysDesc> &v, int nmat, const FacLayout &L) {
    std::vector<lp::BandSys> out;
    size_t i = 0;
    for (const auto &s : v)
        for (int f = 0; f < nmat; ++f, ++i) {
            lp::BandSys b{};
            b.off = s.band_off + (long long)f * s.band_size;
            b.stride = s.band_size;
            b.vec = s.dof_off + (long long)f * s.ndof;
            b.foff = L.off[i];
            b.fstride = 0;
            b.n = s.ndof;
            b.bw = s.bw;
            b.nrhs = 1;
            b.ldf = L.ldf;
            out.push_back(b);
        }
    return out;
}

std::vector<lp::BandSys> solve_list(const std::vector<lp::SysDesc> &v, int nrhs, const FacLayout &L) {
    std::vector<lp::BandSys> out;
    for (size_t j = 0; j < v.size(); ++j) {
        const auto &s = v[j];
        lp::BandSys b{};
        b.off = s.band_off;
        b.stride = s.band_size;
        b.vec = s.dof_off;
        b.foff = L.off[j * nrhs];
        b.fstride = nrhs > 1 ? L.off[j * nrhs + 1] - L.off[j * nrhs] : 0;
        b.n = s.ndof;
        b.bw = s.bw;
        b.nrhs = nrhs;
        b.ldf = L.ldf;
        out.push_back(b);
    }
    return out;
}

double time_at(const lp_ctx *c, int64_t step) { return (double)step * c->prm.dt; }

// solve list that turns nmat factored band matrices of system s into their
// inverses: every right-hand side of matrix f shares its factors (stride 0)
// and column j of the inverse is the solution for the j-th unit vector
std::vector<lp::BandSys> inverse_list(const std::vector<lp::SysDesc> &v, int nmat, const FacLayout &L) {
    std::vector<lp::BandSys> out;
    size_t i = 0;
    for (const auto &s : v) {
        const long long n = s.ndof;
        for (int f = 0; f < nmat; ++f, ++i) {
            lp::BandSys b{};
            b.off = s.band_off + (long long)f * s.band_size;
            b.stride = 0;
            b.vec = (long long)i * n * n;
            b.foff = L.off[i];
            b.fstride = 0;
            b.n = s.ndof;
            b.bw = s.bw;
            b.nrhs = s.ndof;
            b.ldf = L.ldf;
            out.push_back(b);
        }
    }
    return out;
}

std::vector<double> identities(long long n, int nmat) {
    std::vector<double> e((size_t)nmat * n * n, 0.0);
    for (int f = 0; f < nmat; ++f)
        for (long long j = 0; j < n; ++j) e[(size_t)f * n * n + j * n + j] = 1.0;
    return e;
}

// run `sweeps` refinement sweeps (solve, then FP64 residual) on one batch
template <typename T>
lp_status refine_porous(lp_ctx *c, const lp::SysDesc *d_sys, int nsys, int maxnodes, double *part, int *ticket,
                        const lp::BandSys *d_sv, const T *fac, int maxbw, int maxn, double *b, double *x, double *r,
                        int *conv, double *rel, int *sw, long long ndof, int sweeps, double tol, bool timed,
                        hipStream_t st) {
    // x = 0, r = b and the flags were set by the right-hand side kernel
    for (int s = 0; s < sweeps; ++s) {
        {
            StageTimer tm(c, timed ? LP_T_POR_SOLVE : -1, st);
            lp::SolveArgs<T> sa{d_sv, fac, r, x, conv, 3, nullptr, (const T *)c->consts, c->const_one<T>(), (const double *)c->consts};
            if (!lp::launch_band_solve<T>(sa, nsys, 3, maxbw, maxn, c->solve_depth, st)) return fail(LP_ERR_UNSUPPORTED, "bandwidth too large for the solve kernels");
        }
        StageTimer tm(c, timed ? LP_T_POR_RES : -1, st);
        lp::ResidualArgs ra{d_sys, c->d_dof2, x, b, r, conv, rel, sw, tol, nullptr, part, ticket};
        ra.tstride = c->tiles_por;
        ra.co = c->d_co;
        lp::launch_porous_residual_tiled(ra, nsys, c->rblk_por, st);
    }
    return LP_OK;
}

template <typename T>
lp_status refine_oseen(lp_ctx *c, const lp::SysDesc *d_sys, int nsys, int maxnodes, double *part, int *ticket,
                       const lp::BandSys *d_sv, const T *fac, int maxbw, int maxn, const double *W1x, const double *W1y,
                       double *b, double *x, double *r, int *conv, double *rel, int *sw, long long ndof, int sweeps,
                       double tol, const int *skip, bool timed, hipStream_t st) {
    // x = 0, r = b and the flags were set by the right-hand side kernel
    for (int s = 0; s < sweeps; ++s) {
        {
            StageTimer tm(c, timed ? LP_T_OSE_SOLVE : -1, st);
            lp::SolveArgs<T> sa{d_sv, fac, r, x, conv, 1, skip, (const T *)c->consts, c->const_one<T>(), (const double *)c->consts};
            if (!lp::launch_band_solve<T>(sa, nsys, 1, maxbw, maxn, c->solve_depth, st)) return fail(LP_ERR_UNSUPPORTED, "bandwidth too large for the solve kernels");
        }
        StageTimer tm(c, timed ? LP_T_OSE_RES : -1, st);
        lp::OseenApplyArgs<double> ra{};
        ra.co = c->d_co;
        ra.sys = d_sys; ra.cls2 = c->d_cls2; ra.dof2 = c->d_dof2; ra.dof1 = c->d_dof1;
        ra.W1[0] = W1x; ra.W1[1] = W1y;
        ra.x = x; ra.b = b; ra.r = r; ra.band = nullptr;
        ra.conv = conv; ra.relres = rel; ra.sweeps = sw; ra.tol = tol; ra.skip = skip;
        ra.part = part; ra.ticket = ticket; ra.tstride = c->tiles_ose;
        lp::launch_oseen_residual_tiled(ra, nsys, c->rblk_ose, st);
    }
    return LP_OK;
}

// Krylov sweeps on the local Oseen batch: each sweep is one FGMRES(m) cycle
// for the correction d of K d = r (right preconditioning by the strip
// solves), x += d, then the FP64 residual with the convergence test.
template <typename T>
lp_status refine_oseen_krylov(lp_ctx *c, double *part, int *ticket, const double *W1x, const double *W1y, int sweeps,
                              bool timed, hipStream_t st) {
    const int nsys = (int)c->P.ose.size(), nstrip = (int)c->P.strip.size();
    lp::GmresArgs ga{c->d_ose, c->gm_m, c->P.dof_total_ose, c->gm_V, c->gm_Z, c->gm_H, c->gm_cs, c->gm_sn, c->gm_g,
                     c->gm_bn, c->gm_done, c->gm_kd, c->opt.krylov_tol, c->conv_ose, c->gm_tot, c->gm_reorth};
    lp::StripArgs sa{c->d_strip, c->d_strip_parent, c->d_ose, c->d_smap, c->d_sown, c->gm_done, c->s_done, c->s_rs, c->s_zs};
    lp::OseenApplyArgs<double> mv{};
    mv.co = c->d_co;
    mv.sys = c->d_ose; mv.cls2 = c->d_cls2; mv.dof2 = c->d_dof2; mv.dof1 = c->d_dof1;
    mv.W1[0] = W1x; mv.W1[1] = W1y;
    mv.b = nullptr; mv.r = c->gm_w; mv.conv = c->gm_done;
    const long long nt = c->P.dof_total_ose;
    for (int sw = 0; sw < sweeps; ++sw) {
        {
            StageTimer tm(c, timed ? LP_T_OSE_SOLVE : -1, st);
            lp::launch_gm_init(ga, nsys, c->r_ose, c->b_ose, sw == 0, st);
            for (int k = 0; k < c->gm_m; ++k) {
                lp::launch_strip_gather(sa, nstrip, c->gm_V + k * nt, st);
                lp::SolveArgs<T> so{c->d_sv_strip, (const T *)c->fac_strip, c->s_rs, c->s_zs, c->s_done, 1, nullptr,
                                    (const T *)c->consts, c->const_one<T>(), (const double *)c->consts, 1};
                if (!lp::launch_band_solve<T>(so, nstrip, 1, c->maxbw_strip, c->maxn_strip, c->solve_depth, st))
                    return fail(LP_ERR_UNSUPPORTED, "strip bandwidth too large for the solve kernels");
                lp::launch_strip_scatter(sa, nstrip, c->gm_Z + k * nt, st);
                mv.x = c->gm_Z + k * nt;
                lp::launch_oseen_residual_tiled(mv, nsys, c->tiles_ose, st);   // apply mode: no norms, a block per tile
                if (!lp::launch_gm_arnoldi(ga, nsys, c->maxn_ose, k, c->gm_w, st))
                    return fail(LP_ERR_UNSUPPORTED, "local Oseen system too large for the Arnoldi kernel");
            }
            lp::launch_gm_update(ga, nsys, c->x_ose, st);
        }
        StageTimer tm(c, timed ? LP_T_OSE_RES : -1, st);
        lp::OseenApplyArgs<double> ra{};
        ra.co = c->d_co;
        ra.sys = c->d_ose; ra.cls2 = c->d_cls2; ra.dof2 = c->d_dof2; ra.dof1 = c->d_dof1;
        ra.W1[0] = W1x; ra.W1[1] = W1y;
        ra.x = c->x_ose; ra.b = c->b_ose; ra.r = c->r_ose; ra.band = nullptr;
        ra.conv = c->conv_ose; ra.relres = c->rel_ose; ra.sweeps = c->sw_ose; ra.tol = c->opt.ir_tol; ra.skip = nullptr;
        ra.part = part; ra.ticket = ticket; ra.tstride = c->tiles_ose;
        lp::launch_oseen_residual_tiled(ra, nsys, c->rblk_ose, st);
    }
    return LP_OK;
}

template <typename T>
lp_status factor_porous(lp_ctx *c, T *band, T *fac, hipStream_t st) {
    lp::AssembleArgs<T> aa{c->d_por, c->d_dof2, band};
    aa.co = c->d_co;
    lp::launch_porous_assemble<T>(aa, (int)c->P.por.size(), st);
    lp::BandArgs<T> ba{c->d_lu_por, band, fac, c->d_flags, nullptr, (T *)c->lu_dummy, (const T *)c->consts, c->const_one<T>(),
                       c->d_lustat};
    if (!lp::launch_band_lu<T>(ba, 3 * (int)c->P.por.size(), c->maxbw_por, c->lu_variant, st))
        return fail(LP_ERR_UNSUPPORTED, "porous bandwidth exceeds the factorisation kernels");
    return LP_OK;
}

template <typename T>
lp_status local_oseen(lp_ctx *c, hipStream_t st, const LocalScratch &ls) {
    const int nsys = (int)c->P.ose.size();
    const long long nf2 = c->nf2;
    const int o = c->ecur, nw = 1 - c->ecur;
    // right-hand sides of (5.8) and Dirichlet values of the new corrections
    lp::OseenArgs oa{};
    oa.co = c->d_co;
    oa.sys = c->d_ose; oa.cls2 = c->d_cls2; oa.dof2 = c->d_dof2; oa.cls1 = c->d_cls1; oa.dof1 = c->d_dof1;
    const double *pro = c->pro_slot((int)((c->n + 1) % lp_ctx::RING));
    oa.W1[0] = pro; oa.W1[1] = pro + nf2;
    oa.W0[0] = pro + 2 * nf2; oa.W0[1] = pro + 3 * nf2;
    oa.Pp = pro + 5 * nf2;
    oa.ex[0] = c->ex_f[3]; oa.ex[1] = c->ex_f[4];
    for (int cc = 0; cc < 2; ++cc) for (int k = 0; k < 3; ++k) oa.load[cc][k] = c->ld_f[3 + cc][k];
    oa.PF0 = pro + 4 * nf2;
    oa.e_old = c->e2[o]; oa.e_new = c->e2[nw]; oa.e_new1 = c->e1[nw];
    oa.b = c->b_ose;
    oa.ir = lp::IrStart{c->x_ose, c->r_ose, c->conv_ose, c->rel_ose, c->sw_ose};
    oa.tf = c->tf_slot((int)((c->n + 1) % lp_ctx::RING));
    oa.skip = nullptr;
    TRY(seg(c, gkey(G_OSE_RHS, c->n + 1) + c->key_off, st, [&](hipStream_t s) -> lp_status {
        StageTimer tm(c, LP_T_OSE_RHS, s);
        lp::launch_oseen_rhs_tiled(oa, nsys, c->tiles_ose, s);
        return LP_OK;
    }));
    // factors of the operator linearised about Pi_h u_cH^{n+1} (factor stream)
    const int fs = (int)((c->n + 1) % lp_ctx::FSLOTS);
    {
        StageTimer tm(c, LP_T_WAIT_FAC, st);
        HIPCHK(hipStreamWaitEvent(st, c->ev_fac[fs], 0));
    }
    return seg(c, gkey(G_OSE_SOLVE, c->n + 1) + c->key_off, st, [&](hipStream_t s) -> lp_status {
        if (c->krylov)
            TRY(refine_oseen_krylov<T>(c, ls.part_ose, ls.tick_ose, oa.W1[0], oa.W1[1], c->krylov_cycles(), true, s));
        else
            TRY(refine_oseen<T>(c, c->d_ose, nsys, c->nodes_ose, ls.part_ose, ls.tick_ose, c->d_sv_ose, (const T *)c->fac_ose[fs], c->maxbw_ose, c->maxn_ose, oa.W1[0], oa.W1[1], c->b_ose,
                                c->x_ose, c->r_ose, c->conv_ose, c->rel_ose, c->sw_ose, c->P.dof_total_ose, c->opt.max_ir,
                                c->opt.ir_tol, nullptr, true, s));
        StageTimer tm(c, LP_T_MERGE, s);
        lp::FinalizeArgs fa{c->d_ose, c->d_dof2, c->d_dof1, c->x_ose, c->e2[nw], c->e1[nw], nullptr,
                            lp::IrTotals{c->conv_ose, c->sw_ose, c->rel_ose, 1, c->d_flags, c->d_irmax, c->d_irrel}};
        lp::launch_oseen_finalize(fa, nsys, c->nodes_ose, s);
        return LP_OK;
    });
}

void prolong_step(lp_ctx *c, int cnew, int cold, int slot, hipStream_t st);

// Assemble and factor the local Oseen operators of time level m (linearised
// about Pi_h u_cH^m) on factor stream m % 2 (band slot m % 2, ordered by that
// stream), into factor slot m % FSLOTS.  Ordered after coarse step m; the
// factor slot's previous reader, local step m - FSLOTS, is waited for.
template <typename T>
lp_status factor_oseen(lp_ctx *c, int64_t m) {
    const int nw = (int)(m % lp_ctx::RING), bs = (int)(m % 2), fs = (int)(m % lp_ctx::FSLOTS);
    hipStream_t st = c->fstream[bs];
    const int nsys = (int)c->P.ose.size();
    HIPCHK(hipStreamWaitEvent(st, c->ev_coarse[nw], 0));
    // factor slot fs was last read by local step m - FSLOTS
    if (m > lp_ctx::FSLOTS) HIPCHK(hipStreamWaitEvent(st, c->ev_local[(m - lp_ctx::FSLOTS) % lp_ctx::RING], 0));
    T *band = (T *)c->band_ose[bs];
    // the fine-lattice prolongations of level m, for this assembly, the local
    // Oseen stage and the merge of step m; slot nw was last read by local step
    // m - RING, finished before local step m - RING + 1 (coarse step m waited
    // for it)
    TRY(seg(c, gkey(G_PROLONG, m), st, [&](hipStream_t s) -> lp_status {
        StageTimer tm(c, LP_T_PROLONG, s);
        prolong_step(c, nw, (int)((m - 1) % lp_ctx::RING), nw, s);
        return LP_OK;
    }));
    HIPCHK(hipEventRecord(c->ev_pro[nw], st));
    if (c->krylov) {
        // the Krylov path has no per-step factorisation (its strip factors are constant)
        HIPCHK(hipEventRecord(c->ev_fac[fs], st));
        return LP_OK;
    }
    const double *pro_Uf = c->pro_slot(nw);
    TRY(seg(c, gkey(G_FACTOR, m), st, [&](hipStream_t s) -> lp_status {
        {
            StageTimer tm(c, LP_T_OSE_ASM, s);
            // without first writes the band is cleared by a kernel (a memset
            // node would not replay reliably in a graph)
            if (!c->asm_first_write) lp::launch_zero_fill(band, (size_t)c->P.band_total_ose * sizeof(T), s);
            lp::OseenApplyArgs<T> aa{};
            aa.co = c->d_co;
            aa.first_write = c->asm_first_write ? 1 : 0;
            aa.sys = c->d_ose; aa.cls2 = c->d_cls2; aa.dof2 = c->d_dof2; aa.dof1 = c->d_dof1;
            aa.W1[0] = pro_Uf; aa.W1[1] = pro_Uf + c->nf2; aa.band = band;
            lp::launch_oseen_assemble<T>(aa, nsys, c->nodes_ose, s);
        }
        StageTimer tm(c, LP_T_OSE_LU, s);
        lp::BandArgs<T> ba{c->d_lu_ose, band, (T *)c->fac_ose[fs], c->d_flags, nullptr, (T *)c->lu_dummy, (const T *)c->consts,
                           c->const_one<T>(), c->d_lustat};
        if (!lp::launch_band_lu<T>(ba, nsys, c->maxbw_ose, c->lu_variant_ose, s))
            return fail(LP_ERR_UNSUPPORTED, "conduit bandwidth exceeds the factorisation kernels");
        return LP_OK;
    }));
    HIPCHK(hipEventRecord(c->ev_fac[fs], st));
    return LP_OK;
}

// the porous batch's coarse inputs on the batch's stream: p^(n+1), p^n and
// u_y^n prolonged into pro (7 fields)
void prolong_porous(lp_ctx *c, double *pro, int cnew, int cold, hipStream_t st) {
    const long long nc2 = c->nc2, nf2 = c->nf2;
    lp::ProlongArgs pa{};
    pa.NH = c->P.NH; pa.Nh = c->P.Nh; pa.k = c->P.k;
    pa.zs = c->zs;
    pa.nfields = 6;
    for (int f = 0; f < 3; ++f) {
        pa.src[f] = c->cP[cnew] + f * nc2;
        pa.dst[f] = pro + f * nf2;
        pa.src[3 + f] = c->cP[cold] + f * nc2;
        pa.dst[3 + f] = pro + (3 + f) * nf2;
    }
    lp::launch_prolong_p2(pa, c->ns, st);
    pa.nfields = 1;
    pa.src[0] = c->cU[cold] + nc2;
    pa.dst[0] = pro + 6 * nf2;
    lp::launch_prolong_p2(pa, c->ns, st);
}

template <typename T>
lp_status local_porous(lp_ctx *c, const double *pro, hipStream_t st, const LocalScratch &ls) {
    const int nsys = (int)c->P.por.size();
    const long long nf2 = c->nf2;
    const int o = c->ecur, nw = 1 - c->ecur;
    lp::PorousArgs pa{};
    pa.co = c->d_co;
    pa.sys = c->d_por; pa.cls2 = c->d_cls2; pa.dof2 = c->d_dof2;
    for (int f = 0; f < 3; ++f) {
        pa.P1[f] = pro + f * nf2;
        pa.P0[f] = pro + (3 + f) * nf2;
        pa.ex[f] = c->ex_f[f];
        pa.load[f][0] = c->ld_f[f][0];
        pa.load[f][1] = c->ld_f[f][1];
    }
    pa.Uy0 = pro + 6 * nf2;
    pa.e_old = c->e2[o]; pa.e_new = c->e2[nw]; pa.b = c->b_por;
    pa.ir = lp::IrStart{c->x_por, c->r_por, c->conv_por, c->rel_por, c->sw_por};
    pa.tf = c->tf_slot((int)((c->n + 1) % lp_ctx::RING));
    {
        StageTimer tm(c, LP_T_POR_RHS, st);
        lp::launch_porous_rhs_tiled(pa, nsys, c->tiles_por, st);
    }
    TRY(refine_porous<T>(c, c->d_por, nsys, c->nodes_por, ls.part_por, ls.tick_por, c->d_sv_por, (const T *)c->fac_por, c->maxbw_por, c->maxn_por, c->b_por,
                         c->x_por, c->r_por, c->conv_por, c->rel_por, c->sw_por, c->P.dof_total_por, c->opt.max_ir,
                         c->opt.ir_tol, true, st));
    StageTimer tm(c, LP_T_MERGE, st);
    lp::FinalizeArgs fa{c->d_por, c->d_dof2, c->d_dof1, c->x_por, c->e2[nw], nullptr, nullptr,
                        lp::IrTotals{c->conv_por, c->sw_por, c->rel_por, 3, c->d_flags, c->d_irmax, c->d_irrel}};
    lp::launch_porous_finalize(fa, nsys, c->nodes_por, st);
    return LP_OK;
}

// The coarse fields that the assembly, the local Oseen stage and the merge of
// step m read, prolonged into slot `slot`: u^m, u^(m-1), p_F^(m-1) (the Gamma
// terms) on the P2 lattice, p^m on P1.  The porous batch prolongs its own
// inputs.
void prolong_step(lp_ctx *c, int cnew, int cold, int slot, hipStream_t st) {
    const long long nc2 = c->nc2, nf2 = c->nf2;
    double *d = c->pro_slot(slot);
    lp::ProlongArgs pa{};
    pa.NH = c->P.NH; pa.Nh = c->P.Nh; pa.k = c->P.k;
    pa.zs = c->zs;
    pa.nfields = 5;
    for (int cc = 0; cc < 2; ++cc) {
        pa.src[cc] = c->cU[cnew] + cc * nc2;
        pa.dst[cc] = d + cc * nf2;
        pa.src[2 + cc] = c->cU[cold] + cc * nc2;
        pa.dst[2 + cc] = d + (2 + cc) * nf2;
    }
    pa.src[4] = c->cP[cold];
    pa.dst[4] = d + 4 * nf2;
    lp::launch_prolong_p2(pa, c->ns, st);
    pa.nfields = 1;
    pa.src[0] = c->cp[cnew];
    pa.dst[0] = d + 5 * nf2;
    lp::launch_prolong_p1(pa, c->ns, st);
}

// level 0 prolonged for the initial corrections: the three porous pressures
// and the velocity
void prolong_setup(lp_ctx *c, hipStream_t st) {
    const long long nc2 = c->nc2, nf2 = c->nf2;
    lp::ProlongArgs pa{};
    pa.NH = c->P.NH; pa.Nh = c->P.Nh; pa.k = c->P.k;
    pa.zs = c->zs;
    pa.nfields = 5;
    for (int f = 0; f < 3; ++f) {
        pa.src[f] = c->cP[0] + f * nc2;
        pa.dst[f] = c->pro_P1 + f * nf2;
    }
    for (int cc = 0; cc < 2; ++cc) {
        pa.src[3 + cc] = c->cU[0] + cc * nc2;
        pa.dst[3 + cc] = c->pro_U1 + cc * nf2;
    }
    lp::launch_prolong_p2(pa, c->ns, st);
}

// Krylov path: strip tables, the strips' Stokes-part band matrices (the
// local Oseen operator without b_N, constant in time) factored once, and the
// FGMRES work space.
template <typename T>
lp_status setup_strips(lp_ctx *c, hipStream_t st) {
    const lp::Plan &P = c->P;
    const int nstrip = (int)P.strip.size(), nsys = (int)P.ose.size();
    TRY(c->upload(&c->d_strip, P.strip, st));
    TRY(c->upload(&c->d_strip_parent, P.strip_parent, st));
    TRY(c->upload(&c->d_smap, P.smap, st));
    TRY(c->upload(&c->d_sown, P.sown, st));
    const FacLayout fl = fac_layout(P.strip, 1, c->maxbw_strip);
    TRY(c->upload(&c->d_lu_strip, lu_list(P.strip, 1, fl), st));
    TRY(c->upload(&c->d_sv_strip, solve_list(P.strip, 1, fl), st));
    T *band = nullptr, *fac = nullptr;
    TRY(c->dalloc(&band, P.band_total_strip + 64));
    TRY(c->dalloc(&fac, fl.total + 64));
    c->band_strip = band;
    c->fac_strip = fac;
    HIPCHK(hipMemsetAsync(band, 0, (size_t)P.band_total_strip * sizeof(T), st));
    HIPCHK(hipMemsetAsync(fac, 0, (size_t)fl.total * sizeof(T), st));
    lp::OseenApplyArgs<T> aa{};
    aa.co = c->d_co;
    aa.sys = c->d_strip; aa.cls2 = c->d_cls2; aa.dof2 = c->d_dof2; aa.dof1 = c->d_dof1;
    aa.W1[0] = c->pro_U1; aa.W1[1] = c->pro_U1 + c->nf2;   // not read: no convection
    aa.band = band;
    aa.no_convection = 1;
    int nodes = 0;
    for (const auto &s : P.strip) nodes = std::max(nodes, s.lw2 * s.lh2);
    lp::launch_oseen_assemble<T>(aa, nstrip, nodes, st);
    lp::BandArgs<T> ba{c->d_lu_strip, band, fac, c->d_flags, nullptr, (T *)c->lu_dummy, (const T *)c->consts, c->const_one<T>(),
                       c->d_lustat};
    if (!lp::launch_band_lu<T>(ba, nstrip, c->maxbw_strip, c->lu_variant_ose, st))
        return fail(LP_ERR_UNSUPPORTED, "strip bandwidth exceeds the factorisation kernels");
    const long long nt = P.dof_total_ose, m = c->gm_m;
    TRY(c->dalloc(&c->gm_V, (m + 1) * nt));
    TRY(c->dalloc(&c->gm_Z, m * nt));
    TRY(c->dalloc(&c->gm_w, nt));
    TRY(c->dalloc(&c->gm_H, nsys * (m + 1) * m));
    TRY(c->dalloc(&c->gm_cs, nsys * m));
    TRY(c->dalloc(&c->gm_sn, nsys * m));
    TRY(c->dalloc(&c->gm_g, nsys * (m + 1)));
    TRY(c->dalloc(&c->gm_bn, nsys));
    TRY(c->dalloc(&c->gm_done, nsys));
    TRY(c->dalloc(&c->gm_kd, nsys));
    TRY(c->dalloc(&c->gm_tot, nsys));
    HIPCHK(hipMemsetAsync(c->gm_tot, 0, nsys * sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->gm_Z, 0, (size_t)(m * nt) * sizeof(double), st));
    TRY(c->dalloc(&c->s_rs, P.dof_total_strip));
    TRY(c->dalloc(&c->s_zs, P.dof_total_strip));
    TRY(c->dalloc(&c->s_done, nstrip));
    return LP_OK;
}

// milliseconds between two events recorded around fn's launches on st
template <class F>
lp_status time_launches(hipStream_t st, double *ms, F &&fn) {
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, st));
    const lp_status s = fn();
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t;
    return s;
}

// Setup-time autotuning of the local Oseen solves on this run's own systems,
// linearised about the prolonged initial velocity, with the right-hand side
// b = -K x for a fixed smooth x (apply mode of the FP64 residual):
//  - band factorisation kernel (variants 9, 8, 0) and band solve prefetch
//    depth (16, 32, and 64 in FP32), each kept at its fastest;
//  - under LP_AUTO with both paths set up: one batch of local Oseen solves
//    (assembly, factorisation and the refinement sweeps, against the
//    refinement sweeps of the Krylov path) by each, the faster kept.
// Each candidate runs once untimed, then once timed.  Nothing here touches
// the time-stepping state: the band, factor and vector buffers used are
// rewritten by every step.
template <typename T>
lp_status autotune(lp_ctx *c, hipStream_t st) {
    const int nsys = (int)c->P.ose.size();
    const long long nt = c->P.dof_total_ose;
    const double *Wx = c->pro_U1, *Wy = c->pro_U1 + c->nf2;
    lp::launch_fill_pattern(c->x_ose, nt, st);
    {
        lp::OseenApplyArgs<double> mv{};
        mv.co = c->d_co;
        mv.sys = c->d_ose; mv.cls2 = c->d_cls2; mv.dof2 = c->d_dof2; mv.dof1 = c->d_dof1;
        mv.W1[0] = Wx; mv.W1[1] = Wy;
        mv.x = c->x_ose; mv.b = nullptr; mv.r = c->b_ose; mv.conv = nullptr;
        lp::launch_oseen_residual_tiled(mv, nsys, c->tiles_ose, st);   // apply mode: no norms, a block per tile
    }
    // x = 0, r = b, flags cleared: the state a local step's right-hand side kernel leaves
    auto reset = [&]() -> lp_status {
        HIPCHK(hipMemsetAsync(c->x_ose, 0, nt * sizeof(double), st));
        HIPCHK(hipMemcpyAsync(c->r_ose, c->b_ose, nt * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemsetAsync(c->conv_ose, 0, nsys * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->sw_ose, 0, nsys * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->rel_ose, 0, nsys * sizeof(double), st));
        return LP_OK;
    };
    if (c->have_dense) {
        T *band = (T *)c->band_ose[0];
        T *fac = (T *)c->fac_ose[0];
        auto factor = [&](int variant) -> lp_status {
            if (!c->asm_first_write) lp::launch_zero_fill(band, (size_t)c->P.band_total_ose * sizeof(T), st);
            lp::OseenApplyArgs<T> aa{};
            aa.co = c->d_co;
            aa.first_write = c->asm_first_write ? 1 : 0;
            aa.sys = c->d_ose; aa.cls2 = c->d_cls2; aa.dof2 = c->d_dof2; aa.dof1 = c->d_dof1;
            aa.W1[0] = Wx; aa.W1[1] = Wy; aa.band = band;
            lp::launch_oseen_assemble<T>(aa, nsys, c->nodes_ose, st);
            lp::BandArgs<T> ba{c->d_lu_ose, band, fac, c->d_flags, nullptr, (T *)c->lu_dummy, (const T *)c->consts, c->const_one<T>(),
                               c->d_lustat};
            if (!lp::launch_band_lu<T>(ba, nsys, c->maxbw_ose, variant, st)) return fail(LP_ERR_UNSUPPORTED, "factorisation variant");
            return LP_OK;
        };
        double best_lu = 1e30;
        int best_v = c->lu_variant_ose;
        float lustat[4];
        HIPCHK(hipMemcpy(lustat, c->d_lustat, sizeof(lustat), hipMemcpyDeviceToHost));
        for (int v : {9, 8, 0}) {
            double ms = 0.0;
            TRY(factor(v));
            TRY(time_launches(st, &ms, [&] { return factor(v); }));
            int flags = 0;
            HIPCHK(hipMemcpy(&flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost));
            if (flags & 4) {
                // a pivot this kernel's arithmetic cannot take: not a candidate
                flags &= ~4;
                HIPCHK(hipMemcpy(c->d_flags, &flags, sizeof(int), hipMemcpyHostToDevice));
                continue;
            }
            if (ms < best_lu) { best_lu = ms; best_v = v; }
        }
        c->lu_variant_ose = best_v;
        HIPCHK(hipMemcpy(c->d_lustat, lustat, sizeof(lustat), hipMemcpyHostToDevice));
        TRY(factor(best_v));
        double best_sv = 1e30;
        int best_d = c->solve_depth;
        for (int d : {16, 32, 64}) {
            if (d == 64 && sizeof(T) != 4) continue;
            c->solve_depth = d;
            double ms = 0.0;
            for (int rep = 0; rep < 2; ++rep) {
                TRY(reset());
                TRY(time_launches(st, &ms, [&] {
                    return refine_oseen<T>(c, c->d_ose, nsys, c->nodes_ose, c->part_ose, c->tick_ose, c->d_sv_ose, (const T *)fac,
                                           c->maxbw_ose, c->maxn_ose, Wx, Wy, c->b_ose, c->x_ose, c->r_ose, c->conv_ose,
                                           c->rel_ose, c->sw_ose, nt, c->opt.max_ir, c->opt.ir_tol, nullptr, false, st);
                }));
            }
            if (ms < best_sv) { best_sv = ms; best_d = d; }
        }
        c->solve_depth = best_d;
        c->tune_dense_ms = best_lu + best_sv;
    }
    if (c->have_strips) {
        double ms = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
            TRY(reset());
            TRY(time_launches(st, &ms, [&] {
                return refine_oseen_krylov<T>(c, c->part_ose, c->tick_ose, Wx, Wy, c->krylov_cycles(), false, st);
            }));
        }
        c->tune_krylov_ms = ms;
    }
    if (c->have_dense && c->have_strips) c->krylov = c->tune_krylov_ms < c->tune_dense_ms;
    c->tuned = true;
    HIPCHK(hipStreamSynchronize(st));
    return LP_OK;
}

bool params_ok(const lp_params &p, std::string &why) {
    for (int i = 0; i < 3; ++i)
        if (!(p.phi[i] > 0 && p.C[i] > 0 && p.k[i] > 0)) { why = "phi, C and k must be positive"; return false; }
    if (!(p.mu_tilde > 0 && p.rho > 0 && p.eta > 0 && p.nu > 0 && p.dt > 0)) { why = "mu_tilde, rho, eta, nu, dt must be positive"; return false; }
    if (!(p.sigma >= 0 && p.sigma_star >= 0 && p.alpha >= 0)) { why = "sigma, sigma_star, alpha must be non-negative"; return false; }
    return true;
}

}  // namespace

namespace {
// The per-sample field arena: the offsets (doubles) of every field that kernels
// read by lattice position, in one sample's block.
struct ArenaLayout {
    long long cP[lp_ctx::RING], cU[lp_ctx::RING], cp[lp_ctx::RING];
    long long nwt_e, nwt_e1, pro_P1, pro_U1, pro_ring, pro_Pb[2], m_P, m_U, m_p;
    long long ld_f[5][3], ld_c[5][3];
    long long total;
};
ArenaLayout arena_layout(long long nf2, long long nf1, long long nc2, long long nc1, long long pro_stride) {
    ArenaLayout L{};
    long long o = 0;
    auto take = [&](long long n) { const long long at = o; o += (n + 63) / 64 * 64; return at; };
    for (int l = 0; l < lp_ctx::RING; ++l) { L.cP[l] = take(3 * nc2); L.cU[l] = take(2 * nc2); L.cp[l] = take(nc1); }
    L.nwt_e = take(2 * nc2); L.nwt_e1 = take(nc1);
    L.pro_P1 = take(3 * nf2); L.pro_U1 = take(2 * nf2);
    L.pro_ring = take(lp_ctx::RING * pro_stride);
    for (int l = 0; l < 2; ++l) L.pro_Pb[l] = take(7 * nf2);
    L.m_P = take(3 * nf2); L.m_U = take(2 * nf2); L.m_p = take(nf1);
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k) { L.ld_f[f][k] = take(nf2); L.ld_c[f][k] = take(nc2); }
    L.total = o;
    return L;
}

// S copies of a system list (sample s's systems after sample s-1's), their
// per-system buffers laid out sample after sample and their lattice fields in
// sample s's arena block
void replicate_samples(std::vector<lp::SysDesc> &v, int S, long long band_total, long long dof_total,
                       long long e2_total, long long e1_total, long long zs) {
    const size_t n = v.size();
    for (int smp = 1; smp < S; ++smp)
        for (size_t i = 0; i < n; ++i) {
            lp::SysDesc d = v[i];
            d.sample = smp;
            d.zo = smp * zs;
            d.band_off += smp * band_total;
            d.dof_off += smp * dof_total;
            d.e2_off += smp * e2_total;
            d.e1_off += smp * e1_total;
            v.push_back(d);
        }
}

// the coefficients of one parameter sample (Section 3.1 / Algorithm 3)
lp::Coef coefficients(const lp_params &q, int convection) {
    lp::Coef co{};
    for (int i = 0; i < 3; ++i) { co.tau[i] = q.phi[i] * q.C[i] / q.dt; co.kap[i] = q.k[i] / q.mu_tilde; }
    co.sst = q.sigma_star * q.k[1] / q.mu_tilde;
    co.s = q.sigma * q.k[2] / q.mu_tilde;
    co.eta = q.eta; co.nu = q.nu; co.rho = q.rho; co.dt = q.dt;
    co.beta = q.alpha * q.nu / std::sqrt(q.k[0]);
    co.ctau = q.eta * q.nu * q.alpha * std::sqrt(q.k[0]) / q.mu_tilde;
    co.convection = convection;
    return co;
}
}  // namespace

extern "C" {

const char *lp_last_error(void) { return g_err.c_str(); }

static lp_status plan_table(const lp::Plan &P0, int32_t which, int32_t sub, std::vector<int64_t> &v) {
    lp::Plan strips;
    const lp::Plan *pp = &P0;
    if (which == 7) {
        // the Krylov path's strips for a strip width of `sub` cells
        strips = P0;
        std::string why;
        if (!lp::build_strips(strips, sub, 2, 159, why)) return fail(LP_ERR_ARG, why);
        for (size_t i = 0; i < strips.strip.size(); ++i) {
            const lp::SysDesc &S = strips.strip[i];
            const int64_t row[7] = {strips.strip_parent[i], S.x0, S.x0 + S.cx, S.y0, S.y0 + S.cy, S.ndof, S.bw};
            v.insert(v.end(), row, row + 7);
        }
        return LP_OK;
    }
    const lp::Plan &P = *pp;
    const int nsub = (int)(P.por.size() + P.ose.size());
    auto sysof = [&](int s) -> const lp::SysDesc * {
        if (s < 0 || s >= nsub) return nullptr;
        return s < (int)P.por.size() ? &P.por[s] : &P.ose[s - P.por.size()];
    };
    if (which == 0) {
        for (int s = 0; s < nsub; ++s) {
            const lp::SysDesc &S = *sysof(s);
            const auto &cx = P.cuts[S.region][0], &cy = P.cuts[S.region][1];
            int loc = S.region == lp::POROUS ? s : s - (int)P.por.size();
            int kx = loc % P.nsx, ky = loc / P.nsx;
            int64_t row[9] = {S.region, S.x0, S.x0 + S.cx, S.y0, S.y0 + S.cy, cx[kx], cx[kx + 1], cy[ky], cy[ky + 1]};
            v.insert(v.end(), row, row + 9);
        }
    } else if (which >= 1 && which <= 4) {
        // one subdomain, or every subdomain in id order (sub = -1; which = 4
        // then covers the conduit subdomains only)
        const int s0 = sub == -1 ? (which == 4 ? (int)P.por.size() : 0) : sub;
        const int s1 = sub == -1 ? nsub : sub + 1;
        for (int s = s0; s < s1; ++s) {
            const lp::SysDesc *S = sysof(s);
            if (!S) return fail(LP_ERR_ARG, "subdomain id out of range");
            if (which == 4 && S->kind != lp::KIND_OSEEN) return fail(LP_ERR_ARG, "which = 4 needs a conduit subdomain");
            long long n2 = (long long)S->lw2 * S->lh2, n1 = (long long)S->lw1 * S->lh1;
            if (which == 1) for (long long q = 0; q < n2; ++q) v.push_back(P.cls2[S->node_off + q]);
            if (which == 2) for (long long q = 0; q < n1; ++q) v.push_back(P.cls1[S->vert_off + q]);
            if (which == 3) for (long long q = 0; q < n2; ++q) v.push_back(P.dof2[S->node_off + q]);
            if (which == 4) for (long long q = 0; q < n1; ++q) v.push_back(P.dof1[S->vert_off + q]);
        }
    } else if (which == 5) {
        for (int s = 0; s < nsub; ++s) { v.push_back(sysof(s)->ndof); v.push_back(sysof(s)->bw); }
    } else if (which == 6) {
        v = {P.cpor.ndof, P.cpor.bw, P.cns.ndof, P.cns.bw};
    } else {
        return fail(LP_ERR_ARG, "unknown query");
    }
    return LP_OK;
}

lp_status lp_plan_query(const lp_mesh *mesh, const lp_partition *part, int32_t which, int32_t sub, int64_t *out,
                        int64_t len, int64_t *needed) {
    if (!mesh || !part || !needed) return fail(LP_ERR_ARG, "NULL argument");
    lp::Plan P;
    std::string err;
    if (!lp::build_plan(*mesh, *part, P, err)) return fail(LP_ERR_ARG, err);
    std::vector<int64_t> v;
    TRY(plan_table(P, which, sub, v));
    *needed = (int64_t)v.size();
    if (out && len >= (int64_t)v.size()) std::memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return LP_OK;
}

lp_status lp_get_index_map(lp_ctx *c, int32_t which, int32_t sub, int64_t *out, int64_t len, int64_t *needed) {
    if (!c || !needed) return fail(LP_ERR_ARG, "NULL argument");
    std::vector<int64_t> v;
    if (c->ns > 1) {
        // the tables of one sample: every sample shares the partition
        lp::Plan one = c->P;
        one.por.resize(c->np1);
        one.ose.resize(c->no1);
        TRY(plan_table(one, which, sub, v));
    } else {
        TRY(plan_table(c->P, which, sub, v));
    }
    *needed = (int64_t)v.size();
    if (out && len >= (int64_t)v.size()) std::memcpy(out, v.data(), v.size() * sizeof(int64_t));
    return LP_OK;
}

lp_status lp_setup(const lp_mesh *mesh, const lp_partition *part, const lp_params *samples, const lp_options *opt,
                   const lp_allocator *alloc, void *stream, lp_ctx **out) {
    if (!mesh || !part || !samples || !opt || !out) return fail(LP_ERR_ARG, "NULL argument");
    *out = nullptr;
    const lp_params *prm = samples;
    std::string why;
    if (opt->nsamples < 0) return fail(LP_ERR_ARG, "nsamples must be >= 0");
    for (int i = 0; i < std::max(opt->nsamples, 1); ++i)
        if (!params_ok(samples[i], why)) return fail(LP_ERR_ARG, "sample " + std::to_string(i) + ": " + why);
    if (opt->solver < LP_AUTO || opt->solver > LP_KRYLOV) return fail(LP_ERR_ARG, "solver must be LP_AUTO, LP_DENSE or LP_KRYLOV");
    if (opt->coarse_ns != LP_NEWTON && opt->coarse_ns != LP_SEMI_IMPLICIT)
        return fail(LP_ERR_ARG, "coarse_ns must be LP_NEWTON or LP_SEMI_IMPLICIT");
    const int nsam = std::max(opt->nsamples, 1);
    for (int i = 1; i < nsam; ++i)
        if (samples[i].dt != samples[0].dt) return fail(LP_ERR_ARG, "every sample must share dt (one time grid)");
    if (nsam > 1 && (opt->solver == LP_KRYLOV || opt->scheme == LP_ONE_GRID))
        return fail(LP_ERR_UNSUPPORTED, "several samples run the dense local path under Algorithm 3 "
                                        "(LP_KRYLOV and LP_ONE_GRID take one sample)");
    if (opt->solver != LP_DENSE && (opt->max_iter < 1 || opt->max_iter > lp::GM_MAX || !(opt->krylov_tol > 0)))
        return fail(LP_ERR_ARG, "Krylov solves need 1 <= max_iter <= " + std::to_string(lp::GM_MAX) + " and krylov_tol > 0");
    if (opt->coarse_ns == LP_SEMI_IMPLICIT) return fail(LP_ERR_UNSUPPORTED, "the semi-implicit coarse step is not built");
    if (opt->problem != LP_MMS_EX1_2D)
        return fail(LP_ERR_UNSUPPORTED, "lp_setup runs the Example 1 manufactured problem only (the Example-3-type "
                                        "variant runs through lp_mini_setup)");
    if (opt->precision != LP_FP64 && opt->precision != LP_MIXED) return fail(LP_ERR_ARG, "precision must be LP_FP64 or LP_MIXED");
    if (opt->max_ir < 1 || opt->max_newton < 1 || !(opt->ir_tol > 0) || !(opt->newton_tol > 0) || opt->jacobian_every < 0)
        return fail(LP_ERR_ARG, "max_ir, max_newton >= 1 and positive tolerances required");
    if (opt->krylov_cycles < 0 || opt->krylov_cycles > opt->max_ir)
        return fail(LP_ERR_ARG, "krylov_cycles must lie in 0..max_ir");
    if (opt->scheme != LP_TWO_GRID && opt->scheme != LP_ONE_GRID) return fail(LP_ERR_ARG, "scheme must be LP_TWO_GRID or LP_ONE_GRID");
    if (opt->lagged != LP_LAG_OWN && opt->lagged != LP_LAG_MERGED)
        return fail(LP_ERR_ARG, "lagged must be LP_LAG_OWN or LP_LAG_MERGED");
    if (opt->scheme == LP_ONE_GRID && mesh->refine != 1)
        return fail(LP_ERR_ARG, "LP_ONE_GRID (Algorithm 1) runs on one grid: refine must be 1");
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<lp_ctx> c(new lp_ctx());
    HIPCHK(hipGetDevice(&c->device));
    TRY(init_static_scratch(c->device));
    if (!lp::build_plan(*mesh, *part, c->P, why)) return fail(LP_ERR_ARG, why);
    c->prm = *prm;
    c->samples_h.assign(samples, samples + nsam);
    c->opt = *opt;
    c->mixed = opt->precision == LP_MIXED;
    c->one_grid = opt->scheme == LP_ONE_GRID;
    c->lag_merged = opt->lagged == LP_LAG_MERGED;
    c->lu_variant_ose = 9;
    if (const char *v = std::getenv("LP_OSEEN_ASM")) c->asm_first_write = std::atoi(v) != 0;
    if (const char *v = std::getenv("LP_LU_VARIANT")) c->lu_variant = c->lu_variant_ose = c->lu_variant_cns = std::atoi(v);
    if (const char *v = std::getenv("LP_LU_VARIANT_COARSE")) c->lu_variant_cns = std::atoi(v);
    if (const char *v = std::getenv("LP_SOLVE_DEPTH")) c->solve_depth = std::atoi(v);
    if (alloc && alloc->alloc && alloc->free) { c->alloc = *alloc; c->has_alloc = true; }
    lp::Plan &P = c->P;
    for (const auto &s : P.por) { c->maxbw_por = std::max(c->maxbw_por, s.bw); c->maxn_por = std::max(c->maxn_por, s.ndof); }
    for (const auto &s : P.ose) {
        c->maxbw_ose = std::max(c->maxbw_ose, s.bw);
        c->maxn_ose = std::max(c->maxn_ose, s.ndof);
        c->tiles_ose = std::max(c->tiles_ose, lp::residual_tiles(s.cx, s.cy));
    }
    for (const auto &s : P.por) {
        c->nodes_por = std::max(c->nodes_por, s.lw2 * s.lh2);
        c->tiles_por = std::max(c->tiles_por, lp::residual_tiles(s.cx, s.cy));
    }
    for (const auto &s : P.ose) c->nodes_ose = std::max(c->nodes_ose, s.lw2 * s.lh2);
    // residual blocks per box: RESIDUAL_BLOCKS_TARGET in all, no more than
    // the box's tiles, since every block beyond the first of a box ends with
    // a device-scope fence and ticket for the box's norms
    {
        const long long nbox_por = (long long)P.por.size() * std::max(nsam, 1), nbox_ose = (long long)P.ose.size() * std::max(nsam, 1);
        auto per_box = [](long long nbox, int tiles) {
            const long long want = (lp::RESIDUAL_BLOCKS_TARGET + nbox - 1) / std::max(nbox, 1LL);
            return (int)std::max(1LL, std::min<long long>(tiles, want));
        };
        c->rblk_por = per_box(nbox_por, c->tiles_por);
        c->rblk_ose = per_box(nbox_ose, c->tiles_ose);
    }
    if (const char *v = std::getenv("LP_RES_BLOCKS")) {
        const int k = std::max(1, std::atoi(v));
        c->rblk_por = std::min(c->rblk_por, k);
        c->rblk_ose = std::min(c->rblk_ose, k);
    }
    c->nodes_cpor = P.cpor.lw2 * P.cpor.lh2;
    c->nodes_cns = P.cns.lw2 * P.cns.lh2;
    // local Oseen solver: the band factorisation where the half-bandwidth fits
    // its window, else (or on request) the Krylov path
    c->krylov = opt->solver == LP_KRYLOV || (opt->solver == LP_AUTO && c->maxbw_ose >= 160);
    // with autotuning, LP_AUTO sets up both paths where the dense one fits and
    // keeps the faster (measured at the end of setup)
    const bool try_both = opt->autotune && opt->solver == LP_AUTO && c->maxbw_ose < 160 && nsam == 1;
    c->have_dense = !c->krylov || try_both;
    if (nsam > 1 && c->krylov)
        return fail(LP_ERR_UNSUPPORTED, "several samples need the dense local Oseen path (half-bandwidth <= 159)");
    c->ns = nsam;
    c->np1 = (int)P.por.size();
    c->no1 = (int)P.ose.size();
    c->nf2 = (long long)(2 * P.Nh + 1) * (2 * P.Nh + 1);
    c->nf1 = (long long)(P.Nh + 1) * (P.Nh + 1);
    c->nc2 = (long long)(2 * P.NH + 1) * (2 * P.NH + 1);
    c->nc1 = (long long)(P.NH + 1) * (P.NH + 1);
    c->pro_stride = (5 * c->nf2 + c->nf1 + 63) / 64 * 64;
    const ArenaLayout AL = arena_layout(c->nf2, c->nf1, c->nc2, c->nc1, c->pro_stride);
    c->zs = AL.total;
    if (nsam > 1) {
        replicate_samples(P.por, nsam, P.band_total_por, P.dof_total_por, P.e2_total, P.e1_total, c->zs);
        replicate_samples(P.ose, nsam, P.band_total_ose, P.dof_total_ose, P.e2_total, P.e1_total, c->zs);
        P.band_total_por *= nsam; P.band_total_ose *= nsam;
        P.dof_total_por *= nsam; P.dof_total_ose *= nsam;
        P.e2_total *= nsam; P.e1_total *= nsam;
        P.local_dofs *= nsam;
    }
    c->have_strips = c->krylov || try_both;
    // local systems: window 160 (every factorisation kernel); the coarse
    // ones, factored by the vector-unit kernel when wider, up to LU_MAX_BW
    if (std::max(c->maxbw_por, c->krylov ? 0 : c->maxbw_ose) >= 160 || std::max(P.cpor.bw, P.cns.bw) > lp::LU_MAX_BW)
        return fail(LP_ERR_UNSUPPORTED, "half-bandwidth " +
                                            std::to_string(std::max({c->maxbw_por, c->krylov ? 0 : c->maxbw_ose, P.cpor.bw, P.cns.bw})) +
                                            " exceeds the band kernels' window (159 local, " + std::to_string(lp::LU_MAX_BW) + " coarse)");
    if (c->have_strips) {
        int width = 16;
        if (const char *v = std::getenv("LP_KRYLOV_STRIP")) width = std::atoi(v);
        if (!lp::build_strips(P, width, 2, 159, why)) return fail(LP_ERR_UNSUPPORTED, "Krylov strips: " + why);
        for (const auto &s : P.strip) { c->maxbw_strip = std::max(c->maxbw_strip, s.bw); c->maxn_strip = std::max(c->maxn_strip, s.ndof); }
        if (lp::gm_arnoldi_lds(c->maxn_ose) > lp::GM_LDS_MAX)
            return fail(LP_ERR_UNSUPPORTED, "local Oseen system of " + std::to_string(c->maxn_ose) + " unknowns exceeds the Arnoldi kernel's LDS");
        c->gm_m = opt->max_iter;
        if (const char *v = std::getenv("LP_GM_REORTH")) c->gm_reorth = std::atoi(v) != 0;
    }
    // coefficients (Section 3.1 / Algorithm 3), one set per sample
    std::vector<lp::Coef> cos(nsam);
    for (int i = 0; i < nsam; ++i) cos[i] = coefficients(samples[i], opt->convection ? 1 : 0);
    c->co = cos[0];
    lp::build_refdata(c->ref);
    HIPCHK(lp::upload_constants(c->ref, st));
    TRY(c->upload(&c->d_co, cos, st));
    // tables: the coarse systems of every sample (their states and Newton
    // iterates in the sample's arena block)
    std::vector<lp::SysDesc> cp, cn;
    for (int smp = 0; smp < nsam; ++smp) {
        lp::SysDesc a = P.cpor, b = P.cns;
        a.sample = b.sample = smp;
        a.zo = b.zo = smp * c->zs;
        a.band_off += smp * P.cband_por; b.band_off += smp * P.cband_ns;
        a.dof_off += smp * 3LL * P.cpor.ndof; b.dof_off += smp * (long long)P.cns.ndof;
        a.e2_off += smp * c->zs; b.e2_off += smp * c->zs; b.e1_off += smp * c->zs;
        cp.push_back(a);
        cn.push_back(b);
    }
    TRY(c->upload(&c->d_por, P.por, st));
    TRY(c->upload(&c->d_ose, P.ose, st));
    TRY(c->upload(&c->d_cpor, cp, st));
    TRY(c->upload(&c->d_cns, cn, st));
    TRY(c->upload(&c->d_cls2, P.cls2, st));
    TRY(c->upload(&c->d_dof2, P.dof2, st));
    TRY(c->upload(&c->d_cls1, P.cls1, st));
    TRY(c->upload(&c->d_dof1, P.dof1, st));
    const FacLayout fl_por = fac_layout(P.por, 3, c->maxbw_por), fl_ose = fac_layout(P.ose, 1, c->maxbw_ose);
    const FacLayout fl_cpor = fac_layout(cp, 3, P.cpor.bw), fl_cns = fac_layout(cn, 1, P.cns.bw);
    TRY(c->upload(&c->d_lu_por, lu_list(P.por, 3, fl_por), st));
    TRY(c->upload(&c->d_lu_ose, lu_list(P.ose, 1, fl_ose), st));
    TRY(c->upload(&c->d_lu_cpor, lu_list(cp, 3, fl_cpor), st));
    TRY(c->upload(&c->d_lu_cns, lu_list(cn, 1, fl_cns), st));
    TRY(c->upload(&c->d_sv_por, solve_list(P.por, 3, fl_por), st));
    TRY(c->upload(&c->d_sv_ose, solve_list(P.ose, 1, fl_ose), st));
    TRY(c->upload(&c->d_sv_cpor, solve_list(cp, 3, fl_cpor), st));
    TRY(c->upload(&c->d_sv_cns, solve_list(cn, 1, fl_cns), st));
    for (int r = 0; r < 2; ++r)
        for (int ax = 0; ax < 2; ++ax) {
            TRY(c->upload(&c->d_own[r][ax][0], P.own2_lo[r][ax], st));
            TRY(c->upload(&c->d_own[r][ax][1], P.own2_n[r][ax], st));
            TRY(c->upload(&c->d_own[r][ax][2], P.own1_lo[r][ax], st));
            TRY(c->upload(&c->d_own[r][ax][3], P.own1_n[r][ax], st));
        }
    // manufactured data
    TRY(c->dalloc(&c->arena, (long long)nsam * c->zs));
    {
        double *A0 = c->arena;
        for (int l = 0; l < lp_ctx::RING; ++l) { c->cP[l] = A0 + AL.cP[l]; c->cU[l] = A0 + AL.cU[l]; c->cp[l] = A0 + AL.cp[l]; }
        c->nwt_e = A0 + AL.nwt_e; c->nwt_e1 = A0 + AL.nwt_e1;
        c->pro_P1 = A0 + AL.pro_P1; c->pro_U1 = A0 + AL.pro_U1; c->pro_ring = A0 + AL.pro_ring;
        for (int l = 0; l < 2; ++l) c->pro_Pb[l] = A0 + AL.pro_Pb[l];
        c->m_P = A0 + AL.m_P; c->m_U = A0 + AL.m_U; c->m_p = A0 + AL.m_p;
        for (int f = 0; f < 5; ++f)
            for (int k = 0; k < 3; ++k) { c->ld_f[f][k] = A0 + AL.ld_f[f][k]; c->ld_c[f][k] = A0 + AL.ld_c[f][k]; }
    }
    auto put = [&](double *dst0, int smp, const std::vector<double> &v) -> lp_status {
        HIPCHK(hipMemcpyAsync(dst0 + (long long)smp * c->zs, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st));
        return LP_OK;
    };
    {
        std::vector<double> exf[6], exc[6];
        lp::exact_spatial(P.Nh, exf);
        lp::exact_spatial(P.NH, exc);
        for (int f = 0; f < 6; ++f) { TRY(c->upload(&c->ex_f[f], exf[f], st)); TRY(c->upload(&c->ex_c[f], exc[f], st)); }
        // coarse initial data: nodal interpolants at t = 0 (cos 0 = 1), the
        // same for every sample (the exact solution does not depend on the
        // parameters; the sources do)
        std::vector<double> P0(3 * c->nc2), U0(2 * c->nc2);
        for (int f = 0; f < 3; ++f) std::copy(exc[f].begin(), exc[f].end(), P0.begin() + f * c->nc2);
        for (int cc = 0; cc < 2; ++cc) std::copy(exc[3 + cc].begin(), exc[3 + cc].end(), U0.begin() + cc * c->nc2);
        for (int smp = 0; smp < nsam; ++smp) {
            std::vector<double> lf[5][3], lc[5][3];
            lp::source_loads(P.Nh, samples[smp], lf);
            lp::source_loads(P.NH, samples[smp], lc);
            for (int f = 0; f < 5; ++f)
                for (int k = 0; k < 3; ++k) { TRY(put(c->ld_f[f][k], smp, lf[f][k])); TRY(put(c->ld_c[f][k], smp, lc[f][k])); }
            for (int l = 0; l < lp_ctx::RING; ++l) {
                TRY(put(c->cP[l], smp, P0));
                TRY(put(c->cU[l], smp, U0));
                TRY(put(c->cp[l], smp, exc[5]));
            }
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    TRY(c->dalloc(&c->d_done, nsam));
    TRY(c->dalloc(&c->d_its, 2 * nsam));
    TRY(c->dalloc(&c->d_flags, 4));
    TRY(c->dalloc(&c->d_lustat, 4));
    TRY(c->dalloc(&c->tf_dev, 4 * lp_ctx::RING));
    {
        // slot k's first level: the smallest m >= 1 with m = k mod RING
        std::vector<long long> lv(lp_ctx::RING);
        for (int k = 0; k < lp_ctx::RING; ++k) lv[k] = k == 0 ? lp_ctx::RING : k;
        TRY(c->upload(&c->level_dev, lv, st));
    }
    TRY(c->dalloc(&c->d_irmax, 1));
    TRY(c->dalloc(&c->d_irrel, 1));
    HIPCHK(hipMemsetAsync(c->d_flags, 0, 4 * sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->d_lustat, 0, 4 * sizeof(float), st));
    HIPCHK(hipMemsetAsync(c->d_irmax, 0, sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->d_irrel, 0, sizeof(unsigned long long), st));
    HIPCHK(hipMemsetAsync(c->d_its, 0, 2 * nsam * sizeof(int), st));
    {
        // "converged" before the first coarse step (the Newton start reports
        // an unconverged previous step into the flags)
        const std::vector<int> one(nsam, 1);
        HIPCHK(hipMemcpyAsync(c->d_done, one.data(), nsam * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    for (int l = 0; l < 2; ++l) { TRY(c->dalloc(&c->e2[l], P.e2_total)); TRY(c->dalloc(&c->e1[l], P.e1_total)); }
    const size_t tb = c->mixed ? sizeof(float) : sizeof(double);
    {
        void *p;
        if (c->has_alloc) { p = c->alloc.alloc(P.band_total_por * tb + 256, c->alloc.user); }
        else if (hipMalloc(&p, P.band_total_por * tb + 256) != hipSuccess) p = nullptr;
        if (!p) return fail(LP_ERR_ALLOC, "porous band allocation failed");
        c->owned.push_back(p); c->band_por = p;
        for (int l = 0; l < (c->have_dense ? 2 : 0); ++l) {
            if (c->has_alloc) { p = c->alloc.alloc(P.band_total_ose * tb + 256, c->alloc.user); }
            else if (hipMalloc(&p, P.band_total_ose * tb + 256) != hipSuccess) p = nullptr;
            if (!p) return fail(LP_ERR_ALLOC, "conduit band allocation failed");
            c->owned.push_back(p); c->band_ose[l] = p;
            // once: entries outside the matrices' pattern stay zero
            HIPCHK(hipMemsetAsync(p, 0, P.band_total_ose * tb, st));
        }
        if (c->has_alloc) { p = c->alloc.alloc(fl_por.total * tb + 256, c->alloc.user); }
        else if (hipMalloc(&p, fl_por.total * tb + 256) != hipSuccess) p = nullptr;
        if (!p) return fail(LP_ERR_ALLOC, "porous factor allocation failed");
        c->owned.push_back(p); c->fac_por = p;
        HIPCHK(hipMemsetAsync(p, 0, fl_por.total * tb, st));
        for (int l = 0; l < (c->have_dense ? lp_ctx::FSLOTS : 0); ++l) {
            if (c->has_alloc) { p = c->alloc.alloc(fl_ose.total * tb + 256, c->alloc.user); }
            else if (hipMalloc(&p, fl_ose.total * tb + 256) != hipSuccess) p = nullptr;
            if (!p) return fail(LP_ERR_ALLOC, "conduit factor allocation failed");
            c->owned.push_back(p); c->fac_ose[l] = p;
            HIPCHK(hipMemsetAsync(p, 0, fl_ose.total * tb, st));
        }
    }
    {
        const long long nlu = std::max<long long>(std::max<long long>(std::max<long long>(3LL * P.por.size(), (long long)P.ose.size()),
                                                                      (long long)P.strip.size()), 3);
        // local factorisations use the first nlu sinks, the coarse ones (on the
        // coarse stream) the next three
        c->lu_dummy_coarse_off = nlu * lp::LU_DUMMY_PER_SYS;
        TRY(c->dalloc(&c->lu_dummy, (nlu + 3LL * nsam) * lp::LU_DUMMY_PER_SYS));
        std::vector<double> k3(514, 0.0);
        k3[512] = 1.0;
        const float onef = 1.0f;
        std::memcpy(&k3[513], &onef, sizeof(float));
        TRY(c->upload(&c->consts, k3, st));
    }
    TRY(c->dalloc(&c->band_cpor, nsam * P.cband_por));
    TRY(c->dalloc(&c->band_cns, nsam * P.cband_ns));
    // the Jacobian assembly stores whole rows; entries outside the matrix stay zero
    HIPCHK(hipMemsetAsync(c->band_cns, 0, nsam * P.cband_ns * sizeof(double), st));
    TRY(c->dalloc(&c->fac_cpor, fl_cpor.total + 32));
    TRY(c->dalloc(&c->fac_cns, fl_cns.total + 32));
    HIPCHK(hipMemsetAsync(c->fac_cpor, 0, fl_cpor.total * sizeof(double), st));
    HIPCHK(hipMemsetAsync(c->fac_cns, 0, fl_cns.total * sizeof(double), st));
    TRY(c->dalloc(&c->b_por, P.dof_total_por)); TRY(c->dalloc(&c->x_por, P.dof_total_por)); TRY(c->dalloc(&c->r_por, P.dof_total_por));
    TRY(c->dalloc(&c->b_ose, P.dof_total_ose)); TRY(c->dalloc(&c->x_ose, P.dof_total_ose)); TRY(c->dalloc(&c->r_ose, P.dof_total_ose));
    const long long ncp = 3LL * P.cpor.ndof * nsam, ncn = (long long)P.cns.ndof * nsam;
    TRY(c->dalloc(&c->b_cp, ncp)); TRY(c->dalloc(&c->x_cp, ncp)); TRY(c->dalloc(&c->r_cp, ncp));
    TRY(c->dalloc(&c->b_cn, ncn)); TRY(c->dalloc(&c->x_cn, ncn)); TRY(c->dalloc(&c->r_cn, ncn));
    const long long npf = 3LL * P.por.size(), nof = (long long)P.ose.size();
    TRY(c->dalloc(&c->conv_por, npf)); TRY(c->dalloc(&c->rel_por, npf)); TRY(c->dalloc(&c->sw_por, npf));
    TRY(c->dalloc(&c->conv_ose, nof)); TRY(c->dalloc(&c->rel_ose, nof)); TRY(c->dalloc(&c->sw_ose, nof));
    TRY(c->dalloc(&c->conv_cp, 3 * nsam)); TRY(c->dalloc(&c->rel_cp, 3 * nsam)); TRY(c->dalloc(&c->sw_cp, 3 * nsam));
    TRY(c->dalloc(&c->conv_cn, nsam)); TRY(c->dalloc(&c->rel_cn, nsam)); TRY(c->dalloc(&c->sw_cn, nsam));
    {
        auto nb = [](int nodes) { return (long long)lp::node_blocks(nodes); };
        c->scratch_part_por = 2 * npf * std::max<long long>(nb(c->nodes_por), c->tiles_por);
        c->scratch_part_ose = 2 * nof * std::max<long long>(nb(c->nodes_ose), c->tiles_ose);
        TRY(c->dalloc(&c->part_por, c->scratch_part_por)); TRY(c->dalloc(&c->tick_por, npf));
        TRY(c->dalloc(&c->part_ose, c->scratch_part_ose)); TRY(c->dalloc(&c->tick_ose, nof));
        TRY(c->dalloc(&c->part_cp, 2 * 3 * nsam * nb(c->nodes_cpor))); TRY(c->dalloc(&c->tick_cp, 3 * nsam));
        TRY(c->dalloc(&c->part_cn, 2 * nsam * nb(c->nodes_cns))); TRY(c->dalloc(&c->tick_cn, nsam));
        HIPCHK(hipMemsetAsync(c->tick_por, 0, npf * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->tick_ose, 0, nof * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->tick_cp, 0, 3 * nsam * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->tick_cn, 0, nsam * sizeof(int), st));
        TRY(c->dalloc(&c->tick_dn, nsam)); TRY(c->dalloc(&c->tick_dp, nsam));
        HIPCHK(hipMemsetAsync(c->tick_dn, 0, nsam * sizeof(int), st));
        HIPCHK(hipMemsetAsync(c->tick_dp, 0, nsam * sizeof(int), st));
    }
    HIPCHK(hipMemsetAsync(c->sw_ose, 0, nof * sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->sw_por, 0, npf * sizeof(int), st));
    HIPCHK(hipMemsetAsync(c->rel_ose, 0, nof * sizeof(double), st));
    HIPCHK(hipMemsetAsync(c->rel_por, 0, npf * sizeof(double), st));

    // initial corrections e_j^0 = I_h x_0 - Pi_h x_H^0
    c->ecur = 0;
    HIPCHK(hipStreamCreateWithFlags(&c->cstream, hipStreamNonBlocking));
    if (const char *v = std::getenv("LP_SERIAL")) c->serial = std::atoi(v) != 0;
    c->graphs = opt->graphs != 0;
    if (c->graphs) {
        HIPCHK(hipStreamCreateWithFlags(&c->lstream, hipStreamNonBlocking));
    }
    if (c->serial) {
        // diagnostic: every stage on one internal stream, in program order
        c->fstream[0] = c->fstream[1] = c->cstream;
    } else {
        for (int l = 0; l < 2; ++l) HIPCHK(hipStreamCreateWithFlags(&c->fstream[l], hipStreamNonBlocking));
    }
    for (int i = 0; i < lp_ctx::FSLOTS; ++i) HIPCHK(hipEventCreateWithFlags(&c->ev_fac[i], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_por, hipEventDisableTiming));
    for (int i = 0; i < lp_ctx::RING; ++i) {
        HIPCHK(hipEventCreateWithFlags(&c->ev_coarse[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_local[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_cpor[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_pro[i], hipEventDisableTiming));
    }
    prolong_setup(c.get(), st);
    {
        lp::InitArgs ia{};
        ia.sys = c->d_por; ia.cls2 = c->d_cls2;
        for (int f = 0; f < 3; ++f) { ia.ex[f] = c->ex_f[f]; ia.pro[f] = c->pro_P1 + f * c->nf2; }
        ia.e = c->e2[0]; ia.e1 = c->e1[0];
        lp::launch_init_corrections(ia, (int)P.por.size(), st);
        ia.sys = c->d_ose;
        ia.ex[0] = c->ex_f[3]; ia.ex[1] = c->ex_f[4];
        ia.pro[0] = c->pro_U1; ia.pro[1] = c->pro_U1 + c->nf2;
        lp::launch_init_corrections(ia, (int)P.ose.size(), st);
    }
    // constant porous matrices: local (precision of the run) and coarse (FP64)
    if (c->mixed) {
        HIPCHK(hipMemsetAsync(c->band_por, 0, P.band_total_por * sizeof(float), st));
        TRY(factor_porous<float>(c.get(), (float *)c->band_por, (float *)c->fac_por, st));
    } else {
        HIPCHK(hipMemsetAsync(c->band_por, 0, P.band_total_por * sizeof(double), st));
        TRY(factor_porous<double>(c.get(), (double *)c->band_por, (double *)c->fac_por, st));
    }
    if (c->have_strips) {
        if (c->mixed) TRY(setup_strips<float>(c.get(), st));
        else TRY(setup_strips<double>(c.get(), st));
    }
    HIPCHK(hipMemsetAsync(c->band_cpor, 0, c->ns * P.cband_por * sizeof(double), st));
    {
        const int S = c->ns;
        lp::AssembleArgs<double> aa{c->d_cpor, c->d_dof2, c->band_cpor};
        aa.co = c->d_co;
        lp::launch_porous_assemble<double>(aa, S, st);
        lp::BandArgs<double> ba{c->d_lu_cpor, c->band_cpor, c->fac_cpor, c->d_flags, nullptr, c->lu_dummy + c->lu_dummy_coarse_off,
                                (const double *)c->consts, c->const_one<double>(), c->d_lustat + 2};
        if (!lp::launch_band_lu<double>(ba, 3 * S, P.cpor.bw, c->lu_variant, st)) return fail(LP_ERR_UNSUPPORTED, "coarse bandwidth too large");
        // the coarse porous matrices are constant: invert them once
        const long long n = P.cpor.ndof;
        TRY(c->upload(&c->eye_cp, identities(n, 3 * S), st));
        TRY(c->upload(&c->d_iv_cpor, inverse_list(cp, 3, fl_cpor), st));
        TRY(c->dalloc(&c->inv_cp, 3LL * S * n * n));
        HIPCHK(hipMemsetAsync(c->inv_cp, 0, 3LL * S * n * n * sizeof(double), st));
        lp::SolveArgs<double> sa{c->d_iv_cpor, c->fac_cpor, c->eye_cp, c->inv_cp, nullptr, (int)n, nullptr,
                                 (const double *)c->consts, c->const_one<double>(), (const double *)c->consts};
        if (!lp::launch_band_solve<double>(sa, 3 * S, (int)n, P.cpor.bw, (int)n, c->solve_depth, st)) return fail(LP_ERR_UNSUPPORTED, "coarse bandwidth too large");
        const long long m = P.cns.ndof;
        TRY(c->upload(&c->eye_cn, identities(m, S), st));
        TRY(c->upload(&c->d_iv_cns, inverse_list(cn, 1, fl_cns), st));
        TRY(c->dalloc(&c->inv_cn, (long long)S * m * m));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    int flags = 0;
    HIPCHK(hipMemcpy(&flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags & 4) return fail(LP_ERR_NOCONV, "zero or non-finite pivot while factoring the porous matrices");
    if (opt->autotune) {
        if (c->mixed) TRY(autotune<float>(c.get(), st));
        else TRY(autotune<double>(c.get(), st));
    }
    *out = c.release();
    return LP_OK;
}

lp_status lp_coarse_step(lp_ctx *c, void *stream) {
    if (!c) return fail(LP_ERR_ARG, "NULL context");
    if (c->coarse_pending) return fail(LP_ERR_STATE, "lp_local_step must follow the previous lp_coarse_step");
    (void)stream;   // the coarse stage only touches internal state and runs on the context's own stream
    hipStream_t st = c->cstream;
    const int64_t m = c->n + 1;                       // time level produced
    // The porous solves and the Navier-Stokes solve of a coarse step do not
    // read each other (each takes the other's previous level).  Both stay on
    // the coarse stream: on a factor stream the porous part would queue behind
    // the local porous batch of step m - 2 and tie the coarse steps to the
    // local stage.
    hipStream_t ps = st;
    const lp::Plan &P = c->P;
    const int o = (int)((m - 1) % lp_ctx::RING), nw = (int)(m % lp_ctx::RING);
    // slot m % RING was last read by local step m - RING + 1
    if (m >= lp_ctx::RING) {
        HIPCHK(hipStreamWaitEvent(st, c->ev_local[(m - lp_ctx::RING + 1) % lp_ctx::RING], 0));
        HIPCHK(hipStreamWaitEvent(ps, c->ev_local[(m - lp_ctx::RING + 1) % lp_ctx::RING], 0));
    }
    // level n: the porous part reads u^n on Gamma and p^n, the Navier-Stokes
    // part reads p_F^n (level 0 is complete at setup)
    if (m >= 2) {
        HIPCHK(hipStreamWaitEvent(ps, c->ev_coarse[o], 0));
        HIPCHK(hipStreamWaitEvent(ps, c->ev_cpor[o], 0));
        HIPCHK(hipStreamWaitEvent(st, c->ev_cpor[o], 0));
    }
    StageTimer ttot(c, LP_T_COARSE, st);
    const long long nc2 = c->nc2;
    // (5.1)-(5.3): three SPD solves with lagged exchange and lagged u^n on Gamma
    lp::PorousArgs pa{};
    pa.co = c->d_co;
    pa.sys = c->d_cpor; pa.cls2 = c->d_cls2; pa.dof2 = c->d_dof2;
    for (int f = 0; f < 3; ++f) {
        pa.P1[f] = nullptr; pa.P0[f] = nullptr;
        pa.ex[f] = c->ex_c[f];
        pa.load[f][0] = c->ld_c[f][0];
        pa.load[f][1] = c->ld_c[f][1];
    }
    pa.Uy0 = c->cU[o] + nc2;
    pa.e_old = c->cP[o]; pa.e_new = c->cP[nw]; pa.b = c->b_cp;
    pa.tf = c->tf_slot(nw);
    c->seg_m = m;
    TRY(seg(c, gkey(G_CPOR, m), ps, [&](hipStream_t s) -> lp_status {
        // the level's time factors on the device (its ring slot's counter)
        lp::launch_time_level(c->level_dev + nw, lp_ctx::RING, c->prm.dt, c->tf_slot(nw), s);
        lp::launch_porous_rhs(pa, c->ns, c->nodes_cpor, 8, s);
        // the three solves with the explicit inverses, then the node layout
        lp::DensePorousArgs dp{};
        dp.d = lp::DenseArgs{c->inv_cp, c->b_cp, c->x_cp, P.cpor.ndof, nullptr};
        dp.f = lp::FinalizeArgs{c->d_cpor, c->d_dof2, c->d_dof1, c->x_cp, c->cP[nw], nullptr, nullptr};
        dp.ticket = c->tick_dp;
        lp::launch_dense_porous(dp, 3 * c->ns, s);
        return LP_OK;
    }));
    HIPCHK(hipEventRecord(c->ev_cpor[nw], ps));
    // (5.4): Navier-Stokes by Newton from the extrapolation 2 (u^n, p^n) -
    // (u^(n-1), p^(n-1)) (from (u^n, p^n) at the first step); each iteration
    // solves the Oseen system linearised about the current iterate
    // the Jacobian of a refresh step stays in use (its explicit inverse) until
    // the next refresh
    const int jev = c->opt.jacobian_every > 1 ? c->opt.jacobian_every : 1;
    const bool refresh = (m - 1) % jev == 0;
    TRY(seg(c, gkey(refresh ? G_CNS_REFRESH : G_CNS, m), st, [&](hipStream_t s) -> lp_status {
        {
            const int om = (int)((m + lp_ctx::RING - 2) % lp_ctx::RING), omm = (int)((m + lp_ctx::RING - 3) % lp_ctx::RING);
            const bool ex = m >= 2, ex2 = m >= 3;
            lp::NewtonStartArgs ns{c->cU[o], c->cp[o], ex ? c->cU[om] : nullptr, ex ? c->cp[om] : nullptr,
                                   ex2 ? c->cU[omm] : nullptr, ex2 ? c->cp[omm] : nullptr,
                                   c->cU[nw], c->cp[nw], 2 * nc2, c->nc1, c->d_done, c->d_its, nullptr, 0, c->d_flags};
            ns.zs = c->zs;
            lp::launch_newton_start(ns, c->ns, s);
        }
        for (int it = 0; it < c->opt.max_newton; ++it) {
            lp::OseenArgs oa{};
            oa.co = c->d_co;
            oa.sys = c->d_cns; oa.cls2 = c->d_cls2; oa.dof2 = c->d_dof2; oa.cls1 = c->d_cls1; oa.dof1 = c->d_dof1;
            oa.W1[0] = c->cU[nw]; oa.W1[1] = c->cU[nw] + nc2;
            oa.W0[0] = c->cU[o]; oa.W0[1] = c->cU[o] + nc2;
            oa.Pp = c->cp[nw];
            oa.ex[0] = c->ex_c[3]; oa.ex[1] = c->ex_c[4];
            for (int cc = 0; cc < 2; ++cc) for (int k = 0; k < 3; ++k) oa.load[cc][k] = c->ld_c[3 + cc][k];
            oa.PF0 = c->cP[o];
            oa.e_old = nullptr; oa.e_new = c->nwt_e; oa.e_new1 = c->nwt_e1;
            oa.b = c->b_cn;
            oa.tf = c->tf_slot(nw);
            oa.skip = c->d_done;
            lp::launch_oseen_rhs(oa, c->ns, c->nodes_cns, 8, s);
            if (it == 0 && refresh) {
                // Jacobian at the first iterate; later iterations (and steps, up to
                // the next refresh) reuse its inverse, with residuals of the
                // current iterate (chord steps)
                lp::OseenApplyArgs<double> aa{};
                aa.co = c->d_co;
                aa.sys = c->d_cns; aa.cls2 = c->d_cls2; aa.dof2 = c->d_dof2; aa.dof1 = c->d_dof1;
                aa.W1[0] = oa.W1[0]; aa.W1[1] = oa.W1[1]; aa.band = c->band_cns; aa.skip = c->d_done;
                lp::launch_oseen_rows<double>(aa, c->ns, c->nodes_cns, P.cns.bw, s);
                lp::BandArgs<double> ba{c->d_lu_cns, c->band_cns, c->fac_cns, c->d_flags, c->d_done, c->lu_dummy + c->lu_dummy_coarse_off,
                                        (const double *)c->consts, c->const_one<double>(), c->d_lustat + 2};
                if (!lp::launch_band_lu<double>(ba, c->ns, P.cns.bw, c->lu_variant_cns, s)) return fail(LP_ERR_UNSUPPORTED, "coarse bandwidth too large");
                // explicit inverse of the Jacobian: each chord step is then one
                // dense product instead of a serial band solve
                const int n = P.cns.ndof;
                lp::SolveArgs<double> sa{c->d_iv_cns, c->fac_cns, c->eye_cn, c->inv_cn, nullptr, n, c->d_done,
                                         (const double *)c->consts, c->const_one<double>(), (const double *)c->consts, 1};
                if (!lp::launch_band_solve<double>(sa, c->ns, n, P.cns.bw, n, c->solve_depth, s)) return fail(LP_ERR_UNSUPPORTED, "coarse bandwidth too large");
            }
            // chord step: x = J^-1 b, the correction to the node layout and the
            // update with its convergence test, in one launch
            lp::DenseNewtonArgs dn{};
            dn.d = lp::DenseArgs{c->inv_cn, c->b_cn, c->x_cn, P.cns.ndof, c->d_done};
            dn.f = lp::FinalizeArgs{c->d_cns, c->d_dof2, c->d_dof1, c->x_cn, c->nwt_e, c->nwt_e1, c->d_done};
            dn.u = lp::NewtonArgs{c->cU[nw], c->cp[nw], c->nwt_e, c->nwt_e1, nc2, c->nc1, c->d_done, c->d_its, c->opt.newton_tol, c->zs};
            dn.ticket = c->tick_dn;
            lp::launch_dense_newton(dn, c->ns, s);
        }
        return LP_OK;
    }));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev_coarse[nw], st));
    if (!c->one_grid) {
        if (c->mixed) TRY(factor_oseen<float>(c, m));
        else TRY(factor_oseen<double>(c, m));
    }
    HIPCHK(hipGetLastError());
    c->coarse_pending = true;
    return LP_OK;
}

}  // extern "C"

namespace {

// Algorithm 3 Steps 3-4 for one time level; `ls` holds the refinement
// scratch (the context's buffers or the static array), `clear` says whether
// its tickets must be zeroed first (each stream clears the part it uses).
lp_status local_step_impl(lp_ctx *c, void *stream, const LocalScratch &ls, bool clear) {
    if (!c) return fail(LP_ERR_ARG, "NULL context");
    if (!c->coarse_pending) return fail(LP_ERR_STATE, "lp_local_step needs a preceding lp_coarse_step");
    hipStream_t st = (hipStream_t)stream, st_user = st;
    if (c->serial) st = c->cstream;
    const int64_t m = c->n + 1;
    const int o = (int)((m - 1) % lp_ctx::RING), nw = (int)(m % lp_ctx::RING);
    c->seg_m = m;
    c->key_off = clear ? G_NOALLOC : 0;
    if (c->one_grid) {
        // Algorithm 1: the step is complete once the coarse (= fine) step is
        HIPCHK(hipStreamWaitEvent(st, c->ev_coarse[nw], 0));
        HIPCHK(hipStreamWaitEvent(st, c->ev_cpor[nw], 0));
        HIPCHK(hipEventRecord(c->ev_local[m % lp_ctx::RING], st));
        if (st != st_user) HIPCHK(hipStreamWaitEvent(st_user, c->ev_local[m % lp_ctx::RING], 0));
        c->n += 1;
        c->coarse_pending = false;
        return LP_OK;
    }
    {
        StageTimer tm(c, LP_T_WAIT_COARSE, st);
        HIPCHK(hipStreamWaitEvent(st, c->ev_coarse[nw], 0));
        HIPCHK(hipStreamWaitEvent(st, c->ev_cpor[nw], 0));
        HIPCHK(hipStreamWaitEvent(st, c->ev_pro[nw], 0));
    }
    // The porous batch runs from its own prolongation, so it waits for the
    // coarse level, not for the local Oseen chain of the previous step.  It
    // reads the corrections of step m-1 (the previous porous batch) and
    // overwrites the buffers that the merge of step m-2 read.  In the mixed
    // path it runs on the factor stream of this step, beside the local Oseen
    // chain, which has no idle time.  In the FP64 path the factorisation (over
    // twice as long) keeps the factor streams busy while the local Oseen chain
    // waits for it, so the batch runs on this stream, before that wait.
    hipStream_t ps = c->mixed ? c->fstream[m % 2] : st;
    double *pro = c->pro_Pb[m % 2];
    HIPCHK(hipStreamWaitEvent(ps, c->ev_coarse[nw], 0));
    HIPCHK(hipStreamWaitEvent(ps, c->ev_cpor[nw], 0));
    if (m >= 2) HIPCHK(hipStreamWaitEvent(ps, c->ev_por, 0));
    if (m >= 3) HIPCHK(hipStreamWaitEvent(ps, c->ev_local[(m - 2) % lp_ctx::RING], 0));
    TRY(seg(c, gkey(G_POROUS, m) + c->key_off, ps, [&](hipStream_t s) -> lp_status {
        prolong_porous(c, pro, nw, o, s);
        if (clear) lp::launch_zero_ints(ls.tick_por, 3 * (long long)c->P.por.size(), s);
        return c->mixed ? local_porous<float>(c, pro, s, ls) : local_porous<double>(c, pro, s, ls);
    }));
    if (clear) lp::launch_zero_ints(ls.tick_ose, (long long)c->P.ose.size(), st);
    if (c->mixed) TRY(local_oseen<float>(c, st, ls));
    else TRY(local_oseen<double>(c, st, ls));
    HIPCHK(hipEventRecord(c->ev_por, ps));
    {
        StageTimer tm(c, LP_T_WAIT_POR, st);
        HIPCHK(hipStreamWaitEvent(st, c->ev_por, 0));
    }
    const int en = 1 - c->ecur;
    StageTimer tm(c, LP_T_MERGE, st);
    lp::MergeArgs mr[2];
    for (int r = 0; r < 2; ++r) {
        lp::MergeArgs &ma = mr[r];
        ma = lp::MergeArgs{};
        ma.sys = r == lp::POROUS ? c->d_por : c->d_ose;
        ma.nsx = c->P.nsx; ma.N = c->P.Nh; ma.region = r;
        for (int ax = 0; ax < 2; ++ax) {
            ma.own2_lo[ax] = c->d_own[r][ax][0]; ma.own2_n[ax] = c->d_own[r][ax][1];
            ma.own1_lo[ax] = c->d_own[r][ax][2]; ma.own1_n[ax] = c->d_own[r][ax][3];
        }
        if (r == lp::POROUS) {
            for (int f = 0; f < 3; ++f) { ma.base[f] = pro + f * c->nf2; ma.out[f] = c->m_P + f * c->nf2; }
            ma.base1 = nullptr; ma.out1 = nullptr;
        } else {
            const double *pu = c->pro_slot(nw);
            for (int f = 0; f < 2; ++f) { ma.base[f] = pu + f * c->nf2; ma.out[f] = c->m_U + f * c->nf2; }
            ma.base1 = pu + 5 * c->nf2; ma.out1 = c->m_p;
        }
        ma.e2 = c->e2[en]; ma.e1 = c->e1[en];
        ma.cls2 = c->d_cls2;
        ma.e2w = c->e2[en];
        ma.nper = r == lp::POROUS ? c->np1 : c->no1;
        ma.zs = c->zs;
    }
    TRY(seg(c, gkey(G_MERGE, m), st, [&](hipStream_t s) -> lp_status {
        lp::launch_merge(mr[lp::POROUS], mr[lp::CONDUIT], c->ns, s);
        if (c->lag_merged) lp::launch_lag_merged(mr[lp::POROUS], mr[lp::CONDUIT], c->ns, s);
        return LP_OK;
    }));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev_local[m % lp_ctx::RING], st));
    if (st != st_user) HIPCHK(hipStreamWaitEvent(st_user, c->ev_local[m % lp_ctx::RING], 0));
    c->ecur = en;
    c->n += 1;
    c->coarse_pending = false;
    return LP_OK;
}

}  // namespace

namespace {
// device buffers of one diagnostic call, freed on every return path
struct DiagBuffers {
    std::vector<void *> p;
    template <typename T>
    bool get(T **q, size_t count) {
        void *v = nullptr;
        if (hipMalloc(&v, (count > 0 ? count : 1) * sizeof(T)) != hipSuccess) return false;
        p.push_back(v);
        *q = (T *)v;
        return true;
    }
    ~DiagBuffers() {
        for (void *v : p) (void)hipFree(v);
    }
};

template <typename T>
lp_status band_factor_solve(int nsys, int n, int bw, const double *band, const double *rhs, double *x, int variant,
                            int *flags, double *growth, double *pivot_min) {
    const int ld = 2 * bw + 1, nr = lp::solve_nr(bw);
    if (nr == 0 || bw > lp::LU_MAX_BW || ((variant == 8 || variant == 9) && bw > 160))
        return fail(LP_ERR_UNSUPPORTED, "half-bandwidth beyond the factorisation kernels' window");
    const int ldf = 64 * nr;
    const long long nb = (long long)nsys * n * ld, nfac = (long long)nsys * (2LL * n * ldf + n);
    std::vector<lp::BandSys> sys(nsys);
    for (int s = 0; s < nsys; ++s)
        sys[s] = lp::BandSys{(long long)s * n * ld, 0, (long long)s * n, (long long)s * (2LL * n * ldf + n), 0, n, bw, 1, ldf};
    std::vector<T> bt(band, band + nb);
    const T consts[2] = {T(0), T(1)};
    const double zero64 = 0.0;
    DiagBuffers db;
    lp::BandSys *dsys;
    T *dband, *dfac, *ddummy, *dconst;
    double *dr, *dx, *dz;
    int *dflags;
    float *dstat;
    if (!db.get(&dsys, nsys) || !db.get(&dband, nb) || !db.get(&dfac, nfac) ||
        !db.get(&ddummy, (size_t)nsys * lp::LU_DUMMY_PER_SYS) || !db.get(&dconst, 2) || !db.get(&dr, (size_t)nsys * n) ||
        !db.get(&dx, (size_t)nsys * n) || !db.get(&dz, 1) || !db.get(&dflags, 1) || !db.get(&dstat, 2))
        return fail(LP_ERR_ALLOC, "device allocation failed");
    HIPCHK(hipMemcpy(dsys, sys.data(), sys.size() * sizeof(lp::BandSys), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dband, bt.data(), nb * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dconst, consts, sizeof(consts), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dz, &zero64, sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dr, rhs, (size_t)nsys * n * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(dfac, 0, nfac * sizeof(T)));
    HIPCHK(hipMemset(dflags, 0, sizeof(int)));
    HIPCHK(hipMemset(dstat, 0, 2 * sizeof(float)));
    lp::BandArgs<T> ba{dsys, dband, dfac, dflags, nullptr, ddummy, dconst, dconst + 1, dstat};
    if (!lp::launch_band_lu<T>(ba, nsys, bw, variant, nullptr)) return fail(LP_ERR_UNSUPPORTED, "factorisation variant");
    lp::SolveArgs<T> sa{dsys, dfac, dr, dx, nullptr, 1, nullptr, dconst, dconst + 1, dz};
    sa.assign = 1;
    if (!lp::launch_band_solve<T>(sa, nsys, 1, bw, n, 0, nullptr)) return fail(LP_ERR_UNSUPPORTED, "band solve size");
    HIPCHK(hipGetLastError());
    HIPCHK(hipDeviceSynchronize());
    float st[2];
    HIPCHK(hipMemcpy(x, dx, (size_t)nsys * n * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(flags, dflags, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(st, dstat, sizeof(st), hipMemcpyDeviceToHost));
    *growth = st[0];
    *pivot_min = st[1] > 0.f ? 1.0 / st[1] : 1.0;
    return LP_OK;
}
}  // namespace

extern "C" {

lp_status lp_local_step(lp_ctx *c, void *stream) {
    if (!c) return fail(LP_ERR_ARG, "NULL context");
    return local_step_impl(c, stream, LocalScratch{c->part_por, c->part_ose, c->tick_por, c->tick_ose}, false);
}

lp_status lp_local_step_noalloc(lp_ctx *c, void *stream) {
    if (!c) return fail(LP_ERR_ARG, "NULL context");
    const long long need = c->scratch_part_por + c->scratch_part_ose;     // doubles
    const long long need_t = 3LL * (long long)c->P.por.size() + (long long)c->P.ose.size();
    const long long bytes = need * (long long)sizeof(double) + need_t * (long long)sizeof(int);
    if (bytes > LP_NOALLOC_SCRATCH_BYTES)
        return fail(LP_ERR_UNSUPPORTED, "lp_local_step_noalloc needs " + std::to_string(bytes) +
                                            " bytes of scratch; the static array holds " +
                                            std::to_string((long long)LP_NOALLOC_SCRATCH_BYTES));
    unsigned char *base = nullptr;
    TRY(static_scratch(c->device, &base));
    double *d = (double *)base;
    int *t = (int *)(d + need);
    LocalScratch ls{d, d + c->scratch_part_por, t, t + 3 * c->P.por.size()};
    return local_step_impl(c, stream, ls, true);
}

static lp_status locate(lp_ctx *c, int32_t sample, int32_t field, int32_t level, int32_t sub, const double **ptr,
                        int64_t *len) {
    if (field < LP_U || field > LP_PM) return fail(LP_ERR_ARG, "unknown field");
    if (sample < 0 || sample >= c->ns) return fail(LP_ERR_ARG, "sample out of range (the context holds " + std::to_string(c->ns) + ")");
    const int latest = (int)((c->coarse_pending ? c->n + 1 : c->n) % lp_ctx::RING);
    const long long zo = (long long)sample * c->zs;       // the sample's arena block
    if (level == LP_MERGED_FINE) {
        if (field == LP_U) { *ptr = c->m_U + zo; *len = 2 * c->nf2; }
        else if (field == LP_P) { *ptr = c->m_p + zo; *len = c->nf1; }
        else { *ptr = c->m_P + zo + (field - LP_PF) * c->nf2; *len = c->nf2; }
    } else if (level == LP_COARSE) {
        if (field == LP_U) { *ptr = c->cU[latest] + zo; *len = 2 * c->nc2; }
        else if (field == LP_P) { *ptr = c->cp[latest] + zo; *len = c->nc1; }
        else { *ptr = c->cP[latest] + zo + (field - LP_PF) * c->nc2; *len = c->nc2; }
    } else if (level == LP_LOCAL) {
        // sub: a subdomain id of one sample (porous first)
        const int np = c->np1, nsub = np + c->no1;
        if (sub < 0 || sub >= nsub) return fail(LP_ERR_ARG, "subdomain id out of range");
        const lp::SysDesc &S = sub < np ? c->P.por[sample * c->np1 + sub] : c->P.ose[sample * c->no1 + sub - np];
        const long long nl = (long long)S.lw2 * S.lh2;
        const double *e2 = c->e2[c->ecur], *e1 = c->e1[c->ecur];
        if (S.region == lp::POROUS) {
            if (field == LP_U || field == LP_P) return fail(LP_ERR_ARG, "porous subdomains carry p_F, p_f, p_m");
            *ptr = e2 + S.e2_off + (field - LP_PF) * nl; *len = nl;
        } else {
            if (field == LP_U) { *ptr = e2 + S.e2_off; *len = 2 * nl; }
            else if (field == LP_P) { *ptr = e1 + S.e1_off; *len = (long long)S.lw1 * S.lh1; }
            else return fail(LP_ERR_ARG, "conduit subdomains carry u and p");
        }
    } else {
        return fail(LP_ERR_ARG, "unknown level");
    }
    return LP_OK;
}

lp_status lp_get_size(lp_ctx *c, int32_t field, int32_t level, int32_t sub, int64_t *len) {
    if (!c || !len) return fail(LP_ERR_ARG, "NULL argument");
    if (c->one_grid && level == LP_LOCAL) return fail(LP_ERR_STATE, "the one-grid scheme has no local corrections");
    if (c->one_grid && level == LP_MERGED_FINE) level = LP_COARSE;
    const double *p;
    return locate(c, 0, field, level, sub, &p, len);
}

lp_status lp_get_solution(lp_ctx *c, int32_t sample, int32_t field, int32_t level, int32_t sub, double *out,
                          int64_t len, int32_t out_is_device, void *stream) {
    if (!c || !out) return fail(LP_ERR_ARG, "NULL argument");
    if (c->one_grid && level == LP_LOCAL) return fail(LP_ERR_STATE, "the one-grid scheme has no local corrections");
    if (c->one_grid && level == LP_MERGED_FINE) level = LP_COARSE;
    const double *p;
    int64_t n;
    TRY(locate(c, sample, field, level, sub, &p, &n));
    if (len < n) return fail(LP_ERR_ARG, "output buffer too short: need " + std::to_string(n));
    hipStream_t st = (hipStream_t)stream;
    if (level == LP_COARSE) {
        const int latest = (int)((c->coarse_pending ? c->n + 1 : c->n) % lp_ctx::RING);
        if (c->coarse_pending || c->n > 0) {
            HIPCHK(hipStreamWaitEvent(st, c->ev_coarse[latest], 0));
            HIPCHK(hipStreamWaitEvent(st, c->ev_cpor[latest], 0));
        }
    }
    if (out_is_device) {
        HIPCHK(hipMemcpyAsync(out, p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
        HIPCHK(hipMemcpyAsync(out, p, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return LP_OK;
}

// Statistics of the whole context (sample < 0) or of one sample's systems:
// its Newton iterations and convergence, its last-step refinement sweeps and
// residuals; the sticky flag bits 0 and 2, the run-long maxima and the
// factorisation monitor are the context's.
static lp_status stats_impl(lp_ctx *c, int sample, lp_stats *out) {
    HIPCHK(hipDeviceSynchronize());
    std::memset(out, 0, sizeof(*out));
    out->step = c->n;
    out->n_porous = c->np1;
    out->n_conduit = c->no1;
    out->local_dofs = sample < 0 ? c->P.local_dofs : c->P.local_dofs / c->ns;
    out->max_bw = c->P.max_bw;
    int flags = 0, irmax = 0;
    unsigned long long irrel = 0;
    std::vector<int> its(2 * c->ns), done(c->ns);
    HIPCHK(hipMemcpy(its.data(), c->d_its, its.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(done.data(), c->d_done, done.size() * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&irmax, c->d_irmax, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&irrel, c->d_irrel, sizeof(irrel), hipMemcpyDeviceToHost));
    // over the samples asked for: the last step's most Newton iterations, the run's most
    out->flags = flags & 7;
    if (sample >= 0) out->flags &= ~2;             // bit 1 from this sample's Newton status below
    for (int smp = sample < 0 ? 0 : sample; smp < (sample < 0 ? c->ns : sample + 1); ++smp) {
        out->newton_its = std::max(out->newton_its, its[2 * smp]);
        out->newton_its_max = std::max({out->newton_its_max, its[2 * smp], its[2 * smp + 1]});
        if (c->n > 0 && !done[smp]) out->flags |= 2;
    }
    out->ir_sweeps_max = irmax;
    std::memcpy(&out->ir_relres_max, &irrel, sizeof(double));
    std::vector<int> sw(3 * c->P.por.size() + c->P.ose.size());
    std::vector<double> rel(sw.size());
    const size_t np = 3 * c->P.por.size(), no = c->P.ose.size();
    HIPCHK(hipMemcpy(sw.data(), c->sw_por, np * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(sw.data() + np, c->sw_ose, no * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(rel.data(), c->rel_por, np * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(rel.data() + np, c->rel_ose, no * sizeof(double), hipMemcpyDeviceToHost));
    // the systems of one sample: its porous fields, then its conduit boxes
    const size_t pp0 = sample < 0 ? 0 : 3 * (size_t)sample * c->np1, pp1 = sample < 0 ? np : pp0 + 3 * (size_t)c->np1;
    const size_t oo0 = sample < 0 ? 0 : (size_t)sample * c->no1, oo1 = sample < 0 ? no : oo0 + c->no1;
    for (size_t i = 0; i < sw.size(); ++i) {
        if (i < np ? (i < pp0 || i >= pp1) : (i - np < oo0 || i - np >= oo1)) continue;
        out->ir_sweeps = std::max(out->ir_sweeps, sw[i]);
        out->ir_relres = std::max(out->ir_relres, rel[i]);
        if (i < np) {
            out->ir_sweeps_porous = std::max(out->ir_sweeps_porous, sw[i]);
            out->ir_relres_porous = std::max(out->ir_relres_porous, rel[i]);
        } else {
            out->ir_sweeps_oseen = std::max(out->ir_sweeps_oseen, sw[i]);
            out->ir_relres_oseen = std::max(out->ir_relres_oseen, rel[i]);
        }
    }
    out->solver = c->krylov ? LP_KRYLOV : LP_DENSE;
    out->tuned = c->tuned ? 1 : 0;
    out->lu_variant = c->lu_variant_ose;
    out->solve_depth = c->solve_depth;
    out->tune_dense_ms = c->tune_dense_ms;
    out->tune_krylov_ms = c->tune_krylov_ms;
    if (c->krylov) {
        std::vector<int> tot(no);
        HIPCHK(hipMemcpy(tot.data(), c->gm_tot, no * sizeof(int), hipMemcpyDeviceToHost));
        for (int v : tot) out->krylov_its = std::max(out->krylov_its, v);
    }
    {
        float st[4];
        HIPCHK(hipMemcpy(st, c->d_lustat, sizeof(st), hipMemcpyDeviceToHost));
        out->lu_growth_local = st[0];
        out->lu_pivot_local = st[1] > 0.f ? 1.0 / st[1] : 1.0;
        out->lu_growth_coarse = st[2];
        out->lu_pivot_coarse = st[3] > 0.f ? 1.0 / st[3] : 1.0;
    }
    if (out->flags) {
        return fail(LP_ERR_NOCONV, std::string("flags ") + std::to_string(out->flags) +
                                       ": a refinement, a coarse Newton iteration or a pivot check failed in some step so far");
    }
    return LP_OK;
}

lp_status lp_get_stats(lp_ctx *c, lp_stats *out) {
    if (!c || !out) return fail(LP_ERR_ARG, "NULL argument");
    return stats_impl(c, -1, out);
}

lp_status lp_get_sample_stats(lp_ctx *c, int32_t sample, lp_stats *out) {
    if (!c || !out) return fail(LP_ERR_ARG, "NULL argument");
    if (sample < 0 || sample >= c->ns) return fail(LP_ERR_ARG, "sample out of range (the context holds " + std::to_string(c->ns) + ")");
    return stats_impl(c, sample, out);
}

lp_status lp_band_factor_solve(int32_t nsys, int32_t n, int32_t bw, const double *band, const double *rhs, double *x,
                               int32_t precision, int32_t variant, int32_t *flags, double *growth, double *pivot_min) {
    if (nsys < 1 || n < 1 || bw < 0 || bw >= n || !band || !rhs || !x || !flags || !growth || !pivot_min)
        return fail(LP_ERR_ARG, "sizes or NULL arguments");
    if (variant != 0 && variant != 8 && variant != 9) return fail(LP_ERR_ARG, "variant must be 0, 8 or 9");
    if (precision == LP_FP64) return band_factor_solve<double>(nsys, n, bw, band, rhs, x, variant, flags, growth, pivot_min);
    if (precision == LP_MIXED) return band_factor_solve<float>(nsys, n, bw, band, rhs, x, variant, flags, growth, pivot_min);
    return fail(LP_ERR_ARG, "precision must be LP_FP64 or LP_MIXED");
}

lp_status lp_set_timing(lp_ctx *c, uint32_t mask) {
    if (!c) return fail(LP_ERR_ARG, "NULL context");
    for (auto &r : c->recs) {
        (void)hipEventSynchronize(r.b);
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    for (int i = 0; i < LP_T_COUNT; ++i) { c->tms[i] = 0.0; c->tcnt[i] = 0; }
    c->tmask = mask;
    return LP_OK;
}

lp_status lp_get_timing(lp_ctx *c, double *ms, int64_t *launches, int32_t n) {
    if (!c || !ms || !launches || n < 0 || n > LP_T_COUNT) return fail(LP_ERR_ARG, "bad arguments");
    // diagnostic: LP_TRACE=1 prints every timed interval relative to the first one
    const bool trace = std::getenv("LP_TRACE") && !c->recs.empty();
    for (auto &r : c->recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        if (trace) {
            float ta = 0.0f, tb = 0.0f;
            HIPCHK(hipEventElapsedTime(&ta, c->recs[0].a, r.a));
            HIPCHK(hipEventElapsedTime(&tb, c->recs[0].a, r.b));
            std::fprintf(stderr, "LP_TRACE %d %.4f %.4f\n", r.stage, ta, tb);
        }
        c->tms[r.stage] += t;
        c->tcnt[r.stage] += 1;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    for (int i = 0; i < n; ++i) { ms[i] = c->tms[i]; launches[i] = c->tcnt[i]; }
    return LP_OK;
}

namespace {
// A run's state between steps, in the order it is written: a header, every
// sample's parameters, then the device segments below.  The prolonged fields,
// factors and right-hand sides are rebuilt by the next step and not kept.
struct StateHeader {
    char magic[8];
    int64_t n;                         // completed steps
    int32_t ecur, ns, mixed, scheme, jev, lag;
    int64_t Nh, NH, np1, no1, zs, e2_total, e1_total, inv_len, local_dofs;
};
struct Seg { void *dev; size_t bytes; };

std::vector<Seg> state_segments(lp_ctx *c) {
    const int jev = c->opt.jacobian_every > 1 ? c->opt.jacobian_every : 1;
    std::vector<Seg> v;
    v.push_back({c->arena, (size_t)(c->ns * c->zs) * sizeof(double)});      // coarse ring, merged fields, ...
    v.push_back({c->e2[c->ecur], (size_t)c->P.e2_total * sizeof(double)});  // e_j^n (P2 lattices)
    v.push_back({c->e1[c->ecur], (size_t)c->P.e1_total * sizeof(double)});  // e_j^n (pressure, P1)
    if (jev > 1)                                                             // the Jacobian inverse in use
        v.push_back({c->inv_cn, (size_t)(c->ns * c->P.cns.ndof * c->P.cns.ndof) * sizeof(double)});
    v.push_back({c->level_dev, lp_ctx::RING * sizeof(long long)});
    v.push_back({c->tf_dev, 4 * lp_ctx::RING * sizeof(double)});
    v.push_back({c->d_done, (size_t)c->ns * sizeof(int)});
    v.push_back({c->d_its, (size_t)(2 * c->ns) * sizeof(int)});
    v.push_back({c->d_flags, 4 * sizeof(int)});
    v.push_back({c->d_lustat, 4 * sizeof(float)});
    v.push_back({c->d_irmax, sizeof(int)});
    v.push_back({c->d_irrel, sizeof(unsigned long long)});
    return v;
}

size_t pad8(size_t b) { return (b + 7) / 8 * 8; }

StateHeader state_header(lp_ctx *c) {
    StateHeader h{};
    std::memcpy(h.magic, "LPSTATE1", 8);
    h.n = c->n;
    h.ecur = c->ecur;
    h.ns = c->ns;
    h.mixed = c->mixed ? 1 : 0;
    h.scheme = c->one_grid ? LP_ONE_GRID : LP_TWO_GRID;
    h.jev = c->opt.jacobian_every > 1 ? c->opt.jacobian_every : 1;
    h.lag = c->lag_merged ? LP_LAG_MERGED : LP_LAG_OWN;
    h.Nh = c->P.Nh; h.NH = c->P.NH;
    h.np1 = c->np1; h.no1 = c->no1;
    h.zs = c->zs;
    h.e2_total = c->P.e2_total; h.e1_total = c->P.e1_total;
    h.inv_len = h.jev > 1 ? (int64_t)c->ns * c->P.cns.ndof * c->P.cns.ndof : 0;
    h.local_dofs = c->P.local_dofs;
    return h;
}

size_t state_bytes(lp_ctx *c) {
    size_t b = pad8(sizeof(StateHeader)) + pad8(c->samples_h.size() * sizeof(lp_params));
    for (const Seg &g : state_segments(c)) b += pad8(g.bytes);
    return b;
}
}  // namespace

lp_status lp_state_size(lp_ctx *c, int64_t *bytes) {
    if (!c || !bytes) return fail(LP_ERR_ARG, "NULL argument");
    *bytes = (int64_t)state_bytes(c);
    return LP_OK;
}

lp_status lp_save_state(lp_ctx *c, void *buf, int64_t len, void *stream) {
    if (!c || !buf) return fail(LP_ERR_ARG, "NULL argument");
    if (c->coarse_pending) return fail(LP_ERR_STATE, "a coarse step is pending: save between steps");
    const size_t need = state_bytes(c);
    if (len < (int64_t)need) return fail(LP_ERR_ARG, "state buffer too short (" + std::to_string(need) + " bytes needed)");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(hipDeviceSynchronize());                 // every internal stream's work of the last step
    char *p = (char *)buf;
    std::memset(p, 0, need);
    const StateHeader h = state_header(c);
    std::memcpy(p, &h, sizeof(h));
    p += pad8(sizeof(StateHeader));
    std::memcpy(p, c->samples_h.data(), c->samples_h.size() * sizeof(lp_params));
    p += pad8(c->samples_h.size() * sizeof(lp_params));
    for (const Seg &g : state_segments(c)) {
        if (g.bytes) HIPCHK(hipMemcpy(p, g.dev, g.bytes, hipMemcpyDeviceToHost));
        p += pad8(g.bytes);
    }
    return LP_OK;
}

lp_status lp_load_state(lp_ctx *c, const void *buf, int64_t len, void *stream) {
    if (!c || !buf) return fail(LP_ERR_ARG, "NULL argument");
    if (c->coarse_pending) return fail(LP_ERR_STATE, "a coarse step is pending: load between steps");
    if (len < (int64_t)sizeof(StateHeader)) return fail(LP_ERR_ARG, "state buffer too short");
    StateHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "LPSTATE1", 8) != 0) return fail(LP_ERR_ARG, "not a saved state");
    StateHeader mine = state_header(c);
    mine.n = h.n;
    mine.ecur = h.ecur;
    if (std::memcmp(&h, &mine, sizeof(h)) != 0)
        return fail(LP_ERR_ARG, "the state was saved by a context of another mesh, partition, sample count, "
                                "precision, scheme, jacobian_every or lagged reading");
    const char *p = (const char *)buf + pad8(sizeof(StateHeader));
    if (len < (int64_t)(pad8(sizeof(StateHeader)) + c->samples_h.size() * sizeof(lp_params)))
        return fail(LP_ERR_ARG, "state buffer too short");
    if (std::memcmp(p, c->samples_h.data(), c->samples_h.size() * sizeof(lp_params)) != 0)
        return fail(LP_ERR_ARG, "the state was saved with other parameters");
    if (h.n < 0 || (h.ecur != 0 && h.ecur != 1)) return fail(LP_ERR_ARG, "corrupt state header");
    if (len < (int64_t)state_bytes(c)) return fail(LP_ERR_ARG, "state buffer too short");
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(hipDeviceSynchronize());
    c->ecur = h.ecur;                               // the segments name e2/e1[ecur]
    p += pad8(c->samples_h.size() * sizeof(lp_params));
    for (const Seg &g : state_segments(c)) {
        if (g.bytes) HIPCHK(hipMemcpy(g.dev, p, g.bytes, hipMemcpyHostToDevice));
        p += pad8(g.bytes);
    }
    HIPCHK(hipDeviceSynchronize());
    c->n = h.n;
    return LP_OK;
}

void lp_destroy(lp_ctx *c) {
    if (!c) return;
    (void)hipDeviceSynchronize();
    delete c;
}

}  // extern "C"
