// C-ABI layer of liblbmletkf: argument validation, workspace carving, stream
// ordering of the launches and per-stage timing.  Declarations and the
// contract of every entry point are in include/lbmletkf.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbmletkf.h"
#include "common.h"

using namespace lbmletkf;


namespace {

thread_local std::string g_last_error;

lbmletkf_status fail(lbmletkf_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

lbmletkf_status hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return LBMLETKF_EHIP;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t fbuf, force, loc_pt, loc_g, pts, ybar, dY, dvec, K, yf, partial, counters, nodes, gbuf,
        diag_node, diag_fold, total;
};

// Nodes of the observation route grouped by eigenproblem size.
struct Bucket {
    int n;       // instantiated eigenproblem size
    int offset;  // into the device node list
    int count;
    int stream;   // 0: the caller's stream, k > 0: side stream k - 1
    size_t goff;  // offset (doubles) of its per-node G and h in the workspace
};

struct Ctx {
    lbmletkf_lbm_params lbm;
    lbmletkf_obs_params obs;  // obs.points is not kept (device copy in the workspace)
    LbmDims dims;
    int nobs;
    int lmax;
    int route;  // 1 ensemble, 2 observation
    int n_eig;
    std::vector<Bucket> buckets;
    // side streams that run the smaller node groups concurrently with the largest
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {nullptr, nullptr, nullptr};
    std::vector<int> hist;  // nodes per local-point count
    bool has_force;
    bool distinct_points = true;  // no two observation points on one node
    // health checks (lbmletkf_set_checks): Jacobi sweep cap, divergence limit on
    // the analysis spread and RMSE (<= 0: none), check inside every run_cycle
    int max_sweeps = 30;
    double diverge_limit = 0.0;
    bool check_every_cycle = false;
    // precision form: the apply kernels' contractions on BF16 matrix cores
    bool mfma_transform = false;
    char* ws;
    Layout L;
    // arguments of the last misfit forward sweep (its checkpoints feed the
    // reverse sweep)
    struct Fwd {
        bool valid = false;
        const void* f0 = nullptr;
        double cs = 0.0;
        int steps = 0, times = 0;
        const void* work = nullptr;
    } fwd;
    // the reverse sweep recomputes the next interval's states on this stream
    // while the caller's stream runs the current interval's adjoint steps
    // (created at the first backward call)
    hipStream_t rstream = nullptr;
    hipEvent_t rstart = nullptr, rready[2] = {nullptr, nullptr}, rfree[2] = {nullptr, nullptr};
    // per-stage timing
    int profiling = 0;  // 0 off, 1 every launch, 2 per call: forecast steps and analysis
    struct Rec {
        int stage;
        hipEvent_t a, b;
        int launches;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> event_pool;  // events of collected records, reused

    void* fbuf() const { return ws + L.fbuf; }
    int storage() const { return lbm.storage; }
    size_t state_bytes() const {
        return (size_t)dims.nx * dims.ny * 9 * dims.members * state_elem_bytes(lbm.storage);
    }
    const double* force() const {
        return has_force ? reinterpret_cast<const double*>(ws + L.force) : nullptr;
    }
    int* loc_pt() const { return reinterpret_cast<int*>(ws + L.loc_pt); }
    double* loc_g() const { return reinterpret_cast<double*>(ws + L.loc_g); }
    int* pts() const { return reinterpret_cast<int*>(ws + L.pts); }
    double* ybar() const { return reinterpret_cast<double*>(ws + L.ybar); }
    double* dY() const { return reinterpret_cast<double*>(ws + L.dY); }
    double* dvec() const { return reinterpret_cast<double*>(ws + L.dvec); }
    double* K() const { return route == 2 ? reinterpret_cast<double*>(ws + L.K) : nullptr; }
    double* yf() const { return reinterpret_cast<double*>(ws + L.yf); }
    double* partial() const { return reinterpret_cast<double*>(ws + L.partial); }
    int* counters() const { return reinterpret_cast<int*>(ws + L.counters); }
    int* nodes() const { return reinterpret_cast<int*>(ws + L.nodes); }
    double* gbuf() const { return reinterpret_cast<double*>(ws + L.gbuf); }
    double* diag_node() const { return reinterpret_cast<double*>(ws + L.diag_node); }
    double* diag_fold() const { return reinterpret_cast<double*>(ws + L.diag_fold); }
};

// RAII event pair when profiling is on.  `levels`: the profiling levels at
// which this site records (bit 1: every launch, bit 2: per call); `launches`:
// the launches the pair spans.
constexpr int kPerLaunch = 1 << 1, kPerCall = 1 << 2;
struct StageTimer {
    Ctx* c;
    int stage;
    hipStream_t s;
    int launches;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(Ctx* ctx, int st, hipStream_t stream, int levels = kPerLaunch, int n = 1)
        : c(ctx), stage(st), s(stream), launches(n) {
        if (!c->profiling || !((1 << c->profiling) & levels) || n < 1) return;
        a = take();
        b = take();
        if (!a || !b) {
            if (a) c->event_pool.push_back(a);
            if (b) c->event_pool.push_back(b);
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }
    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!c->event_pool.empty()) {
            e = c->event_pool.back();
            c->event_pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
        }
        return e;
    }
    ~StageTimer() {
        if (!a) return;
        (void)hipEventRecord(b, s);
        c->recs.push_back({stage, a, b, launches});
    }
};

lbmletkf_status check_lbm(const lbmletkf_lbm_params* p) {
    if (!p) return fail(LBMLETKF_EINVAL, "lbm params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(LBMLETKF_ESHAPE, "nx and ny must be >= 3");
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 28)
        return fail(LBMLETKF_ESHAPE, "grid too large (nx*ny must be < 2^28)");
    if (p->members < 1 || p->members > 64)
        return fail(LBMLETKF_ESHAPE, "members must be in 1..64");
    if ((int64_t)p->nx * 9 * p->members >= (int64_t)1 << 31)
        return fail(LBMLETKF_ESHAPE, "nx * 9 * members must be < 2^31 (the slots of one lattice row)");
    if (!(p->tau0 > 0.5) || !std::isfinite(p->tau0))
        return fail(LBMLETKF_EINVAL, "tau0 must be finite and > 1/2");
    if (!(p->cs >= 0.0) || !std::isfinite(p->cs)) return fail(LBMLETKF_EINVAL, "cs must be >= 0");
    if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) return fail(LBMLETKF_EINVAL, "mu must be >= 0");
    if (p->storage != LBMLETKF_F64 && p->storage != LBMLETKF_F32_DEV)
        return fail(LBMLETKF_EINVAL, "storage must be LBMLETKF_F64 or LBMLETKF_F32_DEV");
    return LBMLETKF_OK;
}

lbmletkf_status check_obs(const lbmletkf_obs_params* o, const lbmletkf_lbm_params* p) {
    if (!o) return fail(LBMLETKF_EINVAL, "obs params is NULL");
    if (o->n_points < 1 || !o->points) return fail(LBMLETKF_EINVAL, "need >= 1 observation point");
    if (o->nvar != 2 && o->nvar != 3) return fail(LBMLETKF_EINVAL, "nvar must be 2 or 3");
    for (int v = 0; v < o->nvar; ++v)
        if (!(o->sigma[v] > 0.0) || !std::isfinite(o->sigma[v]))
            return fail(LBMLETKF_EINVAL, "sigma must be finite and > 0");
    if (!(o->beta > 0.0) || !std::isfinite(o->beta))
        return fail(LBMLETKF_EINVAL, "beta must be finite and > 0");
    if (std::isnan(o->d_cut)) return fail(LBMLETKF_EINVAL, "d_cut is NaN");
    if (o->route < 0 || o->route > 2) return fail(LBMLETKF_EINVAL, "unknown route");
    for (int k = 0; k < o->n_points; ++k) {
        const int x = o->points[2 * k], y = o->points[2 * k + 1];
        if (x < 0 || x >= p->nx || y < 0 || y >= p->ny)
            return fail(LBMLETKF_EINVAL, "observation point outside the grid");
    }
    if ((int64_t)o->n_points * o->nvar > 16384)
        return fail(LBMLETKF_ESHAPE, "at most 16384 observations");
    return LBMLETKF_OK;
}

bool infinite_cut(double d_cut) { return !(d_cut > 0.0) || std::isinf(d_cut); }

// Number of observation points inside each node's localization support,
// with the same criterion (squared distance < (2 d_cut)^2) as the GPU table
// build; used for sizing and for grouping nodes.  Returns the maximum.
int local_counts(const lbmletkf_lbm_params* p, const lbmletkf_obs_params* o,
                 std::vector<int>* counts) {
    const size_t plane = (size_t)p->nx * p->ny;
    if (counts) counts->assign(plane, 0);
    if (infinite_cut(o->d_cut)) {
        if (counts) counts->assign(plane, o->n_points);
        return o->n_points;
    }
    const double lim = 4.0 * o->d_cut * o->d_cut;
    int best = 0;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            int cnt = 0;
            for (int k = 0; k < o->n_points; ++k) {
                int dx = std::abs(x - o->points[2 * k]), dy = std::abs(y - o->points[2 * k + 1]);
                dx = std::min(dx, p->nx - dx);
                dy = std::min(dy, p->ny - dy);
                if ((double)(dx * dx + dy * dy) < lim) ++cnt;
            }
            if (counts) (*counts)[(size_t)y * p->nx + x] = cnt;
            best = std::max(best, cnt);
        }
    return best;
}

int even_up(int n) { return (n + 1) & ~1; }

// Analysis cost per node in nanoseconds at each instantiated eigenproblem
// size, measured on MI355X (192 x 192 grid, no localization so that every node
// has the same size, FP64 storage; M barely matters on the observation route).
// Only the ratios between entries are used.
double obs_node_cost(int n) {
    switch (n) {
        case 8: return 6;     case 10: return 8;    case 12: return 11;   case 14: return 16;
        case 16: return 19;   case 18: return 28;   case 20: return 32;   case 22: return 56;
        case 24: return 65;   case 26: return 77;   case 28: return 88;   case 30: return 99;
        case 32: return 109;  case 40: return 404;  case 48: return 687;  case 56: return 1064;
        default: return 1466;
    }
}

double ens_node_cost(int n) {
    switch (n) {
        case 8: return 3.0;   case 16: return 15.6; case 24: return 125;
        case 32: return 133;  case 48: return 718;  default: return 1731;
    }
}

// Choose the eigenproblem route and its instantiated size.  AUTO sums the
// per-node cost of each route over the nodes: the observation route sizes each
// node's problem by that node's own local count (counts[i] points), the
// ensemble route solves an M x M problem at every node.
lbmletkf_status choose_route(const lbmletkf_lbm_params* p, const lbmletkf_obs_params* o,
                             const std::vector<int>& counts, int lmax, int* route, int* n) {
    const int nz = o->nvar * lmax;
    const int nE = ens_size_for(even_up(p->members));
    const int nO = obs_size_for(even_up(nz));
    int r = o->route;
    if (r == LBMLETKF_ROUTE_AUTO) {
        if (nO == 0) {
            r = LBMLETKF_ROUTE_ENSEMBLE;
        } else {
            double cost_obs = 0.0;
            for (int c : counts) cost_obs += obs_node_cost(obs_size_for(even_up(o->nvar * c)));
            const double cost_ens = (double)counts.size() * ens_node_cost(nE);
            r = (cost_obs < cost_ens) ? LBMLETKF_ROUTE_OBSERVATION : LBMLETKF_ROUTE_ENSEMBLE;
        }
    }
    const int sz = (r == LBMLETKF_ROUTE_OBSERVATION) ? nO : nE;
    if (sz == 0)
        return fail(LBMLETKF_EUNSUPPORTED,
                    "observation route needs at most 64 local observations per node");
    const int lds = (r == LBMLETKF_ROUTE_OBSERVATION) ? obs_lds_bytes(sz) : ens_lds_bytes(sz, nz);
    if (lds > 160 * 1024)
        return fail(LBMLETKF_EUNSUPPORTED, "too many local observations for the LDS budget");
    *route = r;
    *n = sz;
    return LBMLETKF_OK;
}

// Doubles of per-node G and h the observation route passes between its two
// kernels: (n^2 + n) per node, n the node's eigenproblem size.
size_t gbuf_doubles(const std::vector<int>& counts, int nvar) {
    size_t total = 0;
    for (int c : counts) total += obs_gbuf_doubles(obs_size_for(even_up(nvar * c)), 1);
    return total;
}

Layout make_layout(const lbmletkf_lbm_params* p, const lbmletkf_obs_params* o, int lmax,
                   int route, size_t gbuf) {
    Layout L{};
    const size_t plane = (size_t)p->nx * p->ny;
    const size_t nobs = (size_t)o->n_points * o->nvar;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.fbuf = take(plane * 9 * p->members * state_elem_bytes(p->storage));
    L.force = take(plane * 2 * sizeof(double));
    L.loc_pt = take(plane * std::max(lmax, 1) * sizeof(int));
    L.loc_g = take(plane * std::max(lmax, 1) * sizeof(double));
    L.pts = take((size_t)o->n_points * 2 * sizeof(int));
    L.ybar = take(nobs * sizeof(double));
    L.dY = take(nobs * p->members * sizeof(double));
    L.dvec = take(nobs * sizeof(double));
    L.K = take(route == 2 ? nobs * nobs * sizeof(double) : 0);
    L.yf = take(nobs * p->members * sizeof(double));
    L.partial = take((size_t)diag_blocks_for((int)plane) * 8 * sizeof(double));
    L.counters = take(16 * sizeof(int));
    L.nodes = take(plane * sizeof(int));
    L.gbuf = take(route == 2 ? gbuf * sizeof(double) : 0);
    // run_cycle's diagnostics: per-node records of forecast and analysis, folds
    L.diag_node = take(2 * plane * kDiagFieldCount * sizeof(double));
    L.diag_fold = take((size_t)2 * diag_fold_blocks((int)plane) * kDiagFieldCount * sizeof(double));
    L.total = off;
    return L;
}

// Adjoint workspace of the misfit sweeps.
struct AdjLayout {
    size_t ckpt, seg[2], lam0, lam1, jbuf, kpart, total;
};

AdjLayout make_adj_layout(const lbmletkf_lbm_params* p, int n_points, int steps, int times) {
    AdjLayout L{};
    const size_t plane = (size_t)p->nx * p->ny;
    const size_t sb = plane * 9 * p->members * state_elem_bytes(p->storage);
    const size_t lb = plane * 9 * p->members * sizeof(double);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.ckpt = take(align_up(sb) * times);
    // two sets of the states between checkpoints: the reverse sweep recomputes
    // one interval into one set while the adjoint steps read the other
    L.seg[0] = take(align_up(sb) * (steps - 1));
    L.seg[1] = take(align_up(sb) * (steps - 1));
    L.lam0 = take(lb);
    L.lam1 = take(lb);
    L.jbuf = take((size_t)p->members * n_points * sizeof(double));
    L.kpart = take((size_t)adjoint_partials({p->nx, p->ny, p->members}) * sizeof(double));
    L.total = off;
    return L;
}

// The public handles are opaque: lbmletkf_ctx / lbmletkf_batch are never
// defined, their pointers carry the internal objects.
Ctx* as_ctx(lbmletkf_ctx* c) { return reinterpret_cast<Ctx*>(c); }
lbmletkf_ctx* as_handle(Ctx* c) { return reinterpret_cast<lbmletkf_ctx*>(c); }

void release_streams(Ctx* c) {
    for (int k = 0; k < Ctx::kSide; ++k) {
        if (c->side[k]) (void)hipStreamDestroy(c->side[k]);
        if (c->join[k]) (void)hipEventDestroy(c->join[k]);
        c->side[k] = nullptr;
        c->join[k] = nullptr;
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    c->fork = nullptr;
    if (c->rstream) (void)hipStreamDestroy(c->rstream);
    c->rstream = nullptr;
    for (hipEvent_t* e : {&c->rstart, &c->rready[0], &c->rready[1], &c->rfree[0], &c->rfree[1]}) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
}
hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// The analysis parameters of a context for the state d_f.
AnalysisParams make_params(const Ctx* c, void* d_f) {
    AnalysisParams p{};
    p.f = d_f;
    p.storage = c->storage();
    p.nx = c->dims.nx;
    p.ny = c->dims.ny;
    p.members = c->dims.members;
    p.dY = c->dY();
    p.K = c->K();
    p.dvec = c->dvec();
    p.loc_pt = c->loc_pt();
    p.loc_g = c->loc_g();
    p.lmax = c->lmax;
    p.nvar = c->obs.nvar;
    p.nobs = c->nobs;
    for (int v = 0; v < 3; ++v)
        p.rinv[v] = v < c->obs.nvar ? 1.0 / (c->obs.sigma[v] * c->obs.sigma[v]) : 0.0;
    p.a = (c->dims.members - 1) / c->obs.beta;
    p.sqrt_beta = std::sqrt(c->obs.beta);
    p.max_sweeps = c->max_sweeps;
    p.mfma_transform = c->mfma_transform ? 1 : 0;
    p.eig_fail = c->counters() + 1;
    p.truth_uv = nullptr;
    p.diag_node = nullptr;
    return p;
}

// Waits for the stream, then the health of the analyses since the last check:
// non-finite members in the diagnostics record (16 doubles, forecast then
// analysis; may be NULL), nodes whose eigensolver reached the sweep cap (the
// counter is cleared), the analysis spread or RMSE above the divergence limit.
lbmletkf_status health_check(Ctx* c, const double* d_diag, hipStream_t s) {
    int cnt[2] = {0, 0};
    double dg[16] = {0.0};
    hipError_t e = hipMemcpyAsync(cnt, c->counters(), sizeof(cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && d_diag)
        e = hipMemcpyAsync(dg, d_diag, sizeof(dg), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemsetAsync(c->counters() + 1, 0, sizeof(int), s);
    if (e != hipSuccess) return hip_fail(e, "health check");
    const double nonfinite = dg[2] + dg[8 + 2];
    const int eig = cnt[1];
    char msg[256];
    if (nonfinite > 0.0 || (d_diag && (!std::isfinite(dg[8]) || !std::isfinite(dg[9])))) {
        std::snprintf(msg, sizeof msg,
                      "non-finite ensemble: %.0f forecast and %.0f analysis member-nodes with a "
                      "non-finite density or velocity; %d node eigensolves at the sweep cap",
                      dg[2], dg[8 + 2], eig);
        return fail(LBMLETKF_ENONFINITE, msg);
    }
    if (eig > 0) {
        std::snprintf(msg, sizeof msg,
                      "%d node eigensolves did not converge within %d Jacobi sweeps", eig,
                      c->max_sweeps);
        return fail(LBMLETKF_EEIG, msg);
    }
    if (d_diag && c->diverge_limit > 0.0 &&
        (dg[8] > c->diverge_limit || dg[9] > c->diverge_limit)) {
        std::snprintf(msg, sizeof msg,
                      "analysis RMSE %.6g or spread %.6g above the divergence limit %.6g", dg[8],
                      dg[9], c->diverge_limit);
        return fail(LBMLETKF_EDIVERGED, msg);
    }
    return LBMLETKF_OK;
}

}  // namespace

extern "C" {

const char* lbmletkf_status_string(int32_t st) {
    switch (st) {
        case LBMLETKF_OK: return "ok";
        case LBMLETKF_EINVAL: return "invalid argument";
        case LBMLETKF_ESHAPE: return "unsupported shape";
        case LBMLETKF_EHIP: return "HIP error";
        case LBMLETKF_ENONFINITE: return "non-finite value";
        case LBMLETKF_EDIVERGED: return "filter diverged";
        case LBMLETKF_EEIG: return "eigensolver did not converge";
        case LBMLETKF_EWORKSPACE: return "workspace missing or too small";
        case LBMLETKF_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char* lbmletkf_last_error(void) { return g_last_error.c_str(); }

lbmletkf_status lbmletkf_workspace_bytes(const lbmletkf_lbm_params* lbm,
                                         const lbmletkf_obs_params* obs, size_t* bytes) {
    lbmletkf_status st = check_lbm(lbm);
    if (st) return st;
    if ((st = check_obs(obs, lbm))) return st;
    if (!bytes) return fail(LBMLETKF_EINVAL, "bytes is NULL");
    std::vector<int> counts;
    const int lmax = local_counts(lbm, obs, &counts);
    int route = 0, n = 0;
    if ((st = choose_route(lbm, obs, counts, lmax, &route, &n))) return st;
    *bytes = make_layout(lbm, obs, lmax, route, gbuf_doubles(counts, obs->nvar)).total;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_plan(const lbmletkf_lbm_params* lbm, const lbmletkf_obs_params* obs,
                              int32_t* max_local_points, int32_t* eig_size, int32_t* route) {
    lbmletkf_status st = check_lbm(lbm);
    if (st) return st;
    if ((st = check_obs(obs, lbm))) return st;
    std::vector<int> counts;
    const int lmax = local_counts(lbm, obs, &counts);
    int r = 0, n = 0;
    if ((st = choose_route(lbm, obs, counts, lmax, &r, &n))) return st;
    if (max_local_points) *max_local_points = lmax;
    if (eig_size) *eig_size = n;
    if (route) *route = r;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_create(const lbmletkf_lbm_params* lbm, const lbmletkf_obs_params* obs,
                                const double* d_force, void* d_workspace, size_t bytes,
                                void* stream, lbmletkf_ctx** ctx_out) {
    lbmletkf_status st = check_lbm(lbm);
    if (st) return st;
    if ((st = check_obs(obs, lbm))) return st;
    if (!ctx_out) return fail(LBMLETKF_EINVAL, "ctx_out is NULL");
    *ctx_out = nullptr;
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign))
        return fail(LBMLETKF_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    std::vector<int> counts;
    const int lmax = local_counts(lbm, obs, &counts);
    int route = 0, n = 0;
    if ((st = choose_route(lbm, obs, counts, lmax, &route, &n))) return st;
    Layout L = make_layout(lbm, obs, lmax, route, gbuf_doubles(counts, obs->nvar));
    if (bytes < L.total) return fail(LBMLETKF_EWORKSPACE, "workspace too small");

    Ctx* c = new Ctx();
    c->lbm = *lbm;
    c->obs = *obs;
    c->obs.points = nullptr;
    c->dims = {lbm->nx, lbm->ny, lbm->members};
    c->nobs = obs->n_points * obs->nvar;
    c->lmax = lmax;
    c->route = route;
    c->n_eig = n;
    c->has_force = d_force != nullptr;
    {
        std::vector<char> seen((size_t)lbm->nx * lbm->ny, 0);
        for (int k = 0; k < obs->n_points; ++k) {
            char& v = seen[(size_t)obs->points[2 * k + 1] * lbm->nx + obs->points[2 * k]];
            if (v) c->distinct_points = false;
            v = 1;
        }
    }
    c->ws = reinterpret_cast<char*>(d_workspace);
    c->L = L;
    c->hist.assign(lmax + 1, 0);
    for (int v : counts) c->hist[v] += 1;
    // group the nodes by the eigenproblem size their local count needs
    std::vector<int> order;
    if (route == LBMLETKF_ROUTE_OBSERVATION) {
        std::vector<std::vector<int>> groups(65);
        for (size_t i = 0; i < counts.size(); ++i)
            groups[obs_size_for(even_up(obs->nvar * counts[i]))].push_back((int)i);
        int maxn = 0;
        for (int sz = 0; sz <= 64; ++sz) {
            if (groups[sz].empty()) continue;
            c->buckets.push_back({sz, (int)order.size(), (int)groups[sz].size(), 0, 0});
            order.insert(order.end(), groups[sz].begin(), groups[sz].end());
            maxn = sz;
        }
        c->n_eig = maxn;
        // Spread the groups over the caller's stream and the side streams by
        // longest-processing-time-first on an estimated cost (the Jacobi sweeps
        // grow as N^3 per node, plus a per-node share for the state passes), so
        // no group waits behind another on one stream while the GPU idles.
        auto cost = [](const Bucket& b) { return (double)b.count * ((double)b.n * b.n * b.n + 3000.0); };
        std::stable_sort(c->buckets.begin(), c->buckets.end(),
                         [&](const Bucket& a, const Bucket& b) { return cost(a) > cost(b); });
        double load[1 + Ctx::kSide] = {0.0, 0.0, 0.0, 0.0};
        size_t goff = 0;
        for (Bucket& b : c->buckets) {
            int best = 0;
            for (int k = 1; k <= Ctx::kSide; ++k)
                if (load[k] < load[best]) best = k;
            b.stream = best;
            load[best] += cost(b);
            b.goff = goff;
            goff += obs_gbuf_doubles(b.n, b.count);
        }
    }
    hipStream_t s = as_stream(stream);
    const size_t plane = (size_t)lbm->nx * lbm->ny;
    hipError_t e = hipSuccess;
    if (d_force)
        e = hipMemcpyAsync(c->ws + L.force, d_force, plane * 2 * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->pts(), obs->points, (size_t)obs->n_points * 2 * sizeof(int),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->counters(), 0, 16 * sizeof(int), s);
    if (e == hipSuccess && c->buckets.size() > 1) {
        e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
        for (int k = 0; k < Ctx::kSide && e == hipSuccess; ++k) {
            e = hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[k], hipEventDisableTiming);
        }
    }
    if (e == hipSuccess && !order.empty())
        e = hipMemcpyAsync(c->nodes(), order.data(), order.size() * sizeof(int),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && lmax > 0)
        e = launch_local_table(c->pts(), obs->n_points, obs->d_cut, lmax, lbm->nx, lbm->ny,
                               c->loc_pt(), c->loc_g(), c->counters(), s);
    int overflow = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&overflow, c->counters(), sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release_streams(c);
        delete c;
        return hip_fail(e, "lbmletkf_create");
    }
    if (overflow != 0) {
        release_streams(c);
        delete c;
        return fail(LBMLETKF_EINVAL, "local-observation table overflow");
    }
    *ctx_out = as_handle(c);
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_destroy(lbmletkf_ctx* ctx) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    for (auto& r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    release_streams(c);
    delete c;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_init_equilibrium(lbmletkf_ctx* ctx, const double* d_rho, const double* d_uv,
                                          void* d_f, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_uv || !d_f) return fail(LBMLETKF_EINVAL, "NULL argument");
    hipError_t e = launch_init_equilibrium(d_rho, d_uv, d_f, c->dims, c->storage(), as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "init_equilibrium");
}

lbmletkf_status lbmletkf_import(lbmletkf_ctx* ctx, const double* d_canonical, void* d_f, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_canonical || !d_f) return fail(LBMLETKF_EINVAL, "NULL argument");
    if ((const void*)d_canonical == (const void*)d_f)
        return fail(LBMLETKF_EINVAL, "import cannot run in place");
    hipError_t e = launch_import(d_canonical, d_f, c->dims, c->storage(), as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "import");
}

lbmletkf_status lbmletkf_export(lbmletkf_ctx* ctx, const void* d_f, double* d_canonical, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_canonical || !d_f) return fail(LBMLETKF_EINVAL, "NULL argument");
    if ((const void*)d_canonical == (const void*)d_f)
        return fail(LBMLETKF_EINVAL, "export cannot run in place");
    hipError_t e = launch_export(d_f, d_canonical, c->dims, c->storage(), as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "export");
}

lbmletkf_status lbm_ensemble_step(lbmletkf_ctx* ctx, void* d_f, int32_t nsteps, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(LBMLETKF_EINVAL, "nsteps must be >= 0");
    hipStream_t s = as_stream(stream);
    void* a = d_f;
    void* b = c->fbuf();
    StageTimer all(c, kStageCollide, s, kPerCall, nsteps);
    // pairs of steps in one launch where the ensemble allows it, a single step
    // for an odd remainder
    const bool two = two_step_supported(c->dims, c->storage());
    for (int k = 0; k < nsteps;) {
        const int n = (two && nsteps - k >= 2) ? 2 : 1;
        StageTimer t(c, kStageCollide, s, kPerLaunch, n);
        hipError_t e = n == 2 ? launch_stream_collide2(a, b, c->force(), c->dims, c->lbm.tau0,
                                                       c->lbm.cs, c->lbm.mu, c->storage(), s)
                              : launch_stream_collide(a, b, c->force(), c->dims, c->lbm.tau0,
                                                      c->lbm.cs, c->lbm.mu, c->storage(), s);
        if (e != hipSuccess) return hip_fail(e, "stream_collide");
        std::swap(a, b);
        k += n;
    }
    if (a != d_f) {
        hipError_t e = hipMemcpyAsync(d_f, a, c->state_bytes(), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "ping-pong copy");
    }
    return LBMLETKF_OK;
}

lbmletkf_status observe(lbmletkf_ctx* ctx, const void* d_f, double* d_yf, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_yf) return fail(LBMLETKF_EINVAL, "NULL argument");
    StageTimer t(c, kStageObserve, as_stream(stream));
    hipError_t e = launch_observe(d_f, c->pts(), c->obs.n_points, c->obs.nvar, d_yf, c->dims,
                                  c->storage(), as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "observe");
}

}  // extern "C"

namespace {

// The analysis of letkf_analyze; with diag_node, the analysis kernels also
// write every node's diagnostics record of the forecast and of the analysis.
lbmletkf_status analyze_impl(Ctx* c, void* d_f, const double* d_yf, const double* d_yo,
                             const double* d_truth_uv, double* diag_node, hipStream_t s) {
    {
        StageTimer t(c, kStageStats, s);
        hipError_t e = launch_obs_stats(d_yf, d_yo, c->nobs, c->dims.members, c->ybar(), c->dY(),
                                        c->dvec(), c->K(), c->storage(), s);
        if (e != hipSuccess) return hip_fail(e, "obs_stats");
    }
    AnalysisParams p = make_params(c, d_f);
    p.truth_uv = d_truth_uv;
    p.diag_node = diag_node;
    StageTimer t(c, kStageAnalysis, s, kPerLaunch | kPerCall);
    hipError_t e = hipSuccess;
    if (c->route == LBMLETKF_ROUTE_OBSERVATION) {
        // the largest group on the caller's stream, the others forked onto the
        // side streams after everything queued so far, then joined back
        const int nb = (int)c->buckets.size();
        bool used[Ctx::kSide] = {false, false, false};
        for (const Bucket& b : c->buckets)
            if (b.stream > 0) used[b.stream - 1] = true;
        if (nb > 1) e = hipEventRecord(c->fork, s);
        for (int k = 0; k < Ctx::kSide && e == hipSuccess; ++k)
            if (used[k]) e = hipStreamWaitEvent(c->side[k], c->fork, 0);
        for (int k = 0; k < nb && e == hipSuccess; ++k) {
            const Bucket& b = c->buckets[k];
            hipStream_t sk = b.stream == 0 ? s : c->side[b.stream - 1];
            e = launch_analysis_obs(p, c->nodes() + b.offset, b.count, b.n, c->gbuf() + b.goff,
                                    sk);
        }
        for (int k = 0; k < Ctx::kSide && e == hipSuccess; ++k) {
            if (!used[k]) continue;
            e = hipEventRecord(c->join[k], c->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, c->join[k], 0);
        }
    } else {
        e = launch_analysis_ens(p, c->n_eig, s);
    }
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "analysis");
}

}  // namespace

extern "C" {

lbmletkf_status letkf_analyze(lbmletkf_ctx* ctx, void* d_f, const double* d_yf, const double* d_yo,
                              void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_yf || !d_yo) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (c->dims.members < 2) return fail(LBMLETKF_EINVAL, "analysis needs >= 2 members");
    return analyze_impl(c, d_f, d_yf, d_yo, nullptr, nullptr, as_stream(stream));
}

lbmletkf_status lbmletkf_diagnostics(lbmletkf_ctx* ctx, const void* d_f, const double* d_truth_uv,
                                     double* d_diag, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_diag) return fail(LBMLETKF_EINVAL, "NULL argument");
    StageTimer t(c, kStageDiag, as_stream(stream));
    hipError_t e = launch_diag(d_f, d_truth_uv, c->dims, c->storage(), c->partial(),
                               diag_blocks_for(c->dims.nx * c->dims.ny), d_diag,
                               as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "diagnostics");
}

lbmletkf_status lbmletkf_diagnostics_noalloc(const lbmletkf_lbm_params* lbm, const void* d_f,
                                             const double* d_truth_uv, double* d_diag,
                                             void* stream) {
    lbmletkf_status st = check_lbm(lbm);
    if (st) return st;
    if (!d_f || !d_diag) return fail(LBMLETKF_EINVAL, "NULL argument");
    const int plane = lbm->nx * lbm->ny;
    if (diag_partial_bytes(plane) > kStaticScratchBytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "a grid of %d nodes needs %zu bytes of scratch; the static scratch holds %zu",
                      plane, diag_partial_bytes(plane), kStaticScratchBytes);
        return fail(LBMLETKF_ESHAPE, msg);
    }
    void* scratch = nullptr;
    hipError_t e = static_scratch(&scratch);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    e = launch_diag(d_f, d_truth_uv, {lbm->nx, lbm->ny, lbm->members}, lbm->storage,
                    reinterpret_cast<double*>(scratch), diag_blocks_for(plane), d_diag,
                    as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "diagnostics_noalloc");
}

lbmletkf_status run_cycle(lbmletkf_ctx* ctx, void* d_f, int32_t nsteps, const double* d_yo,
                          const double* d_truth_uv, double* d_diag, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_yo) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (c->dims.members < 2) return fail(LBMLETKF_EINVAL, "analysis needs >= 2 members");
    lbmletkf_status st = lbm_ensemble_step(ctx, d_f, nsteps, stream);
    if (st) return st;
    if ((st = observe(ctx, d_f, c->yf(), stream))) return st;
    hipStream_t s = as_stream(stream);
    if (!d_diag) return analyze_impl(c, d_f, c->yf(), d_yo, nullptr, nullptr, s);
    // diagnostics of the forecast and of the analysis from the analysis kernels'
    // per-node records (they hold each node's forecast and analysis anyway)
    if ((st = analyze_impl(c, d_f, c->yf(), d_yo, d_truth_uv, c->diag_node(), s))) return st;
    {
        StageTimer t(c, kStageDiag, s);
        hipError_t e = launch_diag_nodes_final(c->diag_node(), c->dims.nx * c->dims.ny,
                                               c->diag_fold(), d_diag, d_diag + LBMLETKF_DIAG_LEN, s);
        if (e != hipSuccess) return hip_fail(e, "diagnostics");
    }
    return c->check_every_cycle ? health_check(c, d_diag, s) : LBMLETKF_OK;
}

lbmletkf_status lbmletkf_set_checks(lbmletkf_ctx* ctx, int32_t max_sweeps, double diverge_limit,
                                    int32_t check_every_cycle) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    if (max_sweeps < 1 || max_sweeps > 100) return fail(LBMLETKF_EINVAL, "max_sweeps must be in 1..100");
    if (std::isnan(diverge_limit)) return fail(LBMLETKF_EINVAL, "diverge_limit is NaN");
    if (check_every_cycle != 0 && check_every_cycle != 1)
        return fail(LBMLETKF_EINVAL, "check_every_cycle must be 0 or 1");
    c->max_sweeps = max_sweeps;
    c->diverge_limit = (diverge_limit > 0.0 && std::isfinite(diverge_limit)) ? diverge_limit : 0.0;
    c->check_every_cycle = check_every_cycle != 0;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_set_matrix_core_transform(lbmletkf_ctx* ctx, int32_t enable) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(LBMLETKF_EINVAL, "enable must be 0 or 1");
    if (enable && c->storage() != LBMLETKF_F32_DEV)
        return fail(LBMLETKF_EUNSUPPORTED, "the matrix-core transform is for FP32 storage");
    c->mfma_transform = enable != 0;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_check(lbmletkf_ctx* ctx, const double* d_diag, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    return health_check(c, d_diag, as_stream(stream));
}

lbmletkf_status lbmletkf_energy_spectrum(lbmletkf_ctx* ctx, const void* d_f, double* d_E, int32_t kmax,
                                         void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_E) return fail(LBMLETKF_EINVAL, "NULL argument");
    const int n = c->dims.nx;
    if (c->dims.ny != n) return fail(LBMLETKF_ESHAPE, "the spectrum needs a square grid");
    if (n > 2048) return fail(LBMLETKF_ESHAPE, "the spectrum supports n <= 2048");
    if (kmax < 0 || kmax > n) return fail(LBMLETKF_EINVAL, "kmax must be in 0..n");
    if (spectrum_scratch_bytes(n, c->dims.members) > c->state_bytes())
        return fail(LBMLETKF_EWORKSPACE, "spectrum scratch exceeds the ping-pong buffer");
    if (d_f == c->fbuf()) return fail(LBMLETKF_EINVAL, "d_f is the workspace's own buffer");
    StageTimer t(c, kStageDiag, as_stream(stream));
    hipError_t e = launch_energy_spectrum(d_f, n, c->dims.members, c->storage(), kmax, c->fbuf(),
                                          d_E, as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "energy_spectrum");
}

lbmletkf_status lbmletkf_adjoint_workspace_bytes(const lbmletkf_lbm_params* lbm,
                                                 int32_t n_points, int32_t steps_per_obs,
                                                 int32_t n_times, size_t* bytes) {
    lbmletkf_status st = check_lbm(lbm);
    if (st) return st;
    if (n_points < 1) return fail(LBMLETKF_EINVAL, "n_points must be >= 1");
    if (steps_per_obs < 1 || n_times < 1)
        return fail(LBMLETKF_EINVAL, "steps_per_obs and n_times must be >= 1");
    if (!bytes) return fail(LBMLETKF_EINVAL, "bytes is NULL");
    *bytes = make_adj_layout(lbm, n_points, steps_per_obs, n_times).total;
    return LBMLETKF_OK;
}

namespace {

lbmletkf_status check_misfit_call(Ctx* c, const void* d_f0, double cs, int steps, int times,
                                  const double* d_yo, void* d_work, size_t bytes,
                                  AdjLayout* L) {
    if (!c || !d_f0 || !d_yo) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (steps < 1 || times < 1)
        return fail(LBMLETKF_EINVAL, "steps_per_obs and n_times must be >= 1");
    if (!(cs >= 0.0) || !std::isfinite(cs)) return fail(LBMLETKF_EINVAL, "cs must be >= 0");
    if (!d_work || (reinterpret_cast<uintptr_t>(d_work) % kAlign))
        return fail(LBMLETKF_EWORKSPACE, "adjoint workspace must be non-NULL and 256-byte aligned");
    *L = make_adj_layout(&c->lbm, c->obs.n_points, steps, times);
    if (bytes < L->total) return fail(LBMLETKF_EWORKSPACE, "adjoint workspace too small");
    return LBMLETKF_OK;
}

// State buffers of the misfit sweeps: checkpoint t (t = 0 is f0 itself) and
// intermediate state j (1 <= j < steps) of the segment being (re)computed.
struct Sweep {
    const void* f0;
    char* w;
    AdjLayout L;
    size_t sb;
    const void* ckpt(int t) const { return t == 0 ? f0 : w + L.ckpt + (size_t)(t - 1) * sb; }
    void* ckpt_mut(int t) const { return w + L.ckpt + (size_t)(t - 1) * sb; }
    int set = 0;  // which of the two sets of intermediate states
    void* seg(int j) const { return w + L.seg[set] + (size_t)(j - 1) * sb; }
    Sweep with_set(int k) const {
        Sweep o = *this;
        o.set = k;
        return o;
    }
};

// Steps 1 .. last of the segment that starts at checkpoint t - 1, every state
// kept; step `steps` (if last == steps) lands in checkpoint t.  Pairs of steps
// run in one launch that also writes the pair's first state, where the
// ensemble allows it (the same bits as single steps).
lbmletkf_status segment_steps(Ctx* c, const Sweep& sw, int t, int steps, int last, double cs,
                              hipStream_t s) {
    const bool two = two_step_supported(c->dims, c->storage());
    for (int j = 1; j <= last;) {
        const void* in = j == 1 ? sw.ckpt(t - 1) : sw.seg(j - 1);
        hipError_t e;
        if (two && j + 1 <= last) {
            void* out = j + 1 == steps ? sw.ckpt_mut(t) : sw.seg(j + 1);
            StageTimer tm(c, kStageCollide, s, kPerLaunch, 2);
            e = launch_stream_collide2(in, out, c->force(), c->dims, c->lbm.tau0, cs, c->lbm.mu,
                                       c->storage(), s, sw.seg(j));
            j += 2;
        } else {
            void* out = j == steps ? sw.ckpt_mut(t) : sw.seg(j);
            StageTimer tm(c, kStageCollide, s);
            e = launch_stream_collide(in, out, c->force(), c->dims, c->lbm.tau0, cs, c->lbm.mu,
                                      c->storage(), s);
            j += 1;
        }
        if (e != hipSuccess) return hip_fail(e, "stream_collide");
    }
    return LBMLETKF_OK;
}

// The whole segment from checkpoint t - 1 to checkpoint t when its
// intermediate states are not kept: pairs of steps in one launch where the
// ensemble allows it (the same bits as single steps), a single step for an
// odd remainder; states in between pass through the segment buffers.
lbmletkf_status segment_advance(Ctx* c, const Sweep& sw, int t, int steps, double cs,
                                hipStream_t s) {
    const bool two = two_step_supported(c->dims, c->storage());
    const void* in = sw.ckpt(t - 1);
    for (int j = 0; j < steps;) {
        const int n = (two && steps - j >= 2) ? 2 : 1;
        void* out = j + n == steps ? sw.ckpt_mut(t) : sw.seg(j + n);
        StageTimer tm(c, kStageCollide, s, kPerLaunch, n);
        hipError_t e = n == 2 ? launch_stream_collide2(in, out, c->force(), c->dims, c->lbm.tau0,
                                                       cs, c->lbm.mu, c->storage(), s)
                              : launch_stream_collide(in, out, c->force(), c->dims, c->lbm.tau0,
                                                      cs, c->lbm.mu, c->storage(), s);
        if (e != hipSuccess) return hip_fail(e, "stream_collide");
        in = out;
        j += n;
    }
    return LBMLETKF_OK;
}

}  // namespace

lbmletkf_status lbmletkf_misfit_forward(lbmletkf_ctx* ctx, const void* d_f0, double cs,
                                        int32_t steps_per_obs, int32_t n_times,
                                        const double* d_yo, double* d_J, void* d_work,
                                        size_t work_bytes, void* stream) {
    Ctx* c = as_ctx(ctx);
    AdjLayout L;
    lbmletkf_status st =
        check_misfit_call(c, d_f0, cs, steps_per_obs, n_times, d_yo, d_work, work_bytes, &L);
    if (st) return st;
    if (!d_J) return fail(LBMLETKF_EINVAL, "NULL argument");
    c->fwd.valid = false;
    hipStream_t s = as_stream(stream);
    Sweep sw{d_f0, reinterpret_cast<char*>(d_work), L, align_up(c->state_bytes())};
    double* jbuf = reinterpret_cast<double*>(sw.w + L.jbuf);
    const size_t nj = (size_t)c->dims.members * c->obs.n_points;
    hipError_t e = launch_fill(jbuf, nj, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "fill");
    for (int t = 1; t <= n_times; ++t) {
        if ((st = segment_advance(c, sw, t, steps_per_obs, cs, s))) return st;
        StageTimer tm(c, kStageMisfit, s);
        e = launch_misfit(sw.ckpt(t), c->pts(), c->obs.n_points, c->obs.nvar,
                          d_yo + (size_t)(t - 1) * c->nobs, nullptr, jbuf, c->dims, c->storage(),
                          s);
        if (e != hipSuccess) return hip_fail(e, "misfit");
    }
    e = launch_sum(jbuf, nj, 1.0, d_J, s);
    if (e != hipSuccess) return hip_fail(e, "sum");
    c->fwd = {true, d_f0, cs, steps_per_obs, n_times, d_work};
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_misfit_backward(lbmletkf_ctx* ctx, const void* d_f0, double cs,
                                         int32_t steps_per_obs, int32_t n_times,
                                         const double* d_yo, void* d_work, size_t work_bytes,
                                         double* d_grad_f0, double* d_grad_cs, void* stream) {
    Ctx* c = as_ctx(ctx);
    AdjLayout L;
    lbmletkf_status st =
        check_misfit_call(c, d_f0, cs, steps_per_obs, n_times, d_yo, d_work, work_bytes, &L);
    if (st) return st;
    if (!d_grad_f0) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (!c->distinct_points)
        return fail(LBMLETKF_EUNSUPPORTED, "the misfit gradient needs distinct observation points");
    const Ctx::Fwd& fw = c->fwd;
    if (!fw.valid || fw.f0 != d_f0 || fw.cs != cs || fw.steps != steps_per_obs ||
        fw.times != n_times || fw.work != d_work)
        return fail(LBMLETKF_EINVAL,
                    "call lbmletkf_misfit_forward with the same arguments before the backward sweep");
    const size_t nlam = (size_t)c->dims.members * 9 * c->dims.nx * c->dims.ny;
    {
        const char* g0 = reinterpret_cast<const char*>(d_grad_f0);
        const char* g1 = g0 + nlam * sizeof(double);
        const char* w0 = reinterpret_cast<const char*>(d_work);
        const char* f0 = reinterpret_cast<const char*>(d_f0);
        if ((g0 < w0 + work_bytes && w0 < g1) || (g0 < f0 + c->state_bytes() && f0 < g1))
            return fail(LBMLETKF_EINVAL, "d_grad_f0 overlaps d_f0 or the workspace");
    }
    hipStream_t s = as_stream(stream);
    Sweep sw{d_f0, reinterpret_cast<char*>(d_work), L, align_up(c->state_bytes())};
    double* cur = reinterpret_cast<double*>(sw.w + L.lam0);
    double* oth = reinterpret_cast<double*>(sw.w + L.lam1);
    double* kpart = reinterpret_cast<double*>(sw.w + L.kpart);
    const int nparts = adjoint_partials(c->dims);
    hipError_t e = launch_fill(cur, nlam, 0.0, s);
    if (e == hipSuccess) e = launch_fill(kpart, (size_t)nparts, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "fill");
    // The states between checkpoints t - 1 and t are recomputed on the
    // recompute stream into set t % 2, one interval ahead of the adjoint steps
    // on the caller's stream: interval t - 1 is recomputed while interval t is
    // reversed, set (t - 1) % 2 being reused once interval t + 1's adjoint
    // steps are done with it.  Same kernels and inputs, so the same bits.
    if (!c->rstream) {
        e = hipStreamCreateWithFlags(&c->rstream, hipStreamNonBlocking);
        for (hipEvent_t* ev : {&c->rstart, &c->rready[0], &c->rready[1], &c->rfree[0], &c->rfree[1]})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_streams(c);
            return hip_fail(e, "recompute stream");
        }
    }
    hipStream_t rs = c->rstream;
    e = hipEventRecord(c->rstart, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(rs, c->rstart, 0);
    if (e != hipSuccess) return hip_fail(e, "recompute fork");
    auto recompute = [&](int t) -> lbmletkf_status {
        if (t + 2 <= n_times) {
            // set t % 2 was last read by interval t + 2's adjoint steps
            hipError_t ee = hipStreamWaitEvent(rs, c->rfree[t % 2], 0);
            if (ee != hipSuccess) return hip_fail(ee, "recompute wait");
        }
        lbmletkf_status r = segment_steps(c, sw.with_set(t % 2), t, steps_per_obs,
                                          steps_per_obs - 1, cs, rs);
        if (r) return r;
        hipError_t ee = hipEventRecord(c->rready[t % 2], rs);
        return ee == hipSuccess ? LBMLETKF_OK : hip_fail(ee, "recompute record");
    };
    if ((st = recompute(n_times))) return st;
    for (int t = n_times; t >= 1; --t) {
        if (t > 1 && (st = recompute(t - 1))) return st;
        const Sweep cw = sw.with_set(t % 2);
        {
            // lam^(t s) += dJ_t/df at the observation nodes
            StageTimer tm(c, kStageMisfit, s);
            e = launch_misfit(sw.ckpt(t), c->pts(), c->obs.n_points, c->obs.nvar,
                              d_yo + (size_t)(t - 1) * c->nobs, cur, nullptr, c->dims,
                              c->storage(), s);
            if (e != hipSuccess) return hip_fail(e, "misfit");
        }
        // the states between checkpoints t - 1 and t
        e = hipStreamWaitEvent(s, c->rready[t % 2], 0);
        if (e != hipSuccess) return hip_fail(e, "recompute join");
        for (int j = steps_per_obs - 1; j >= 0; --j) {
            const void* state = j == 0 ? sw.ckpt(t - 1) : cw.seg(j);
            StageTimer tm(c, kStageAdjoint, s);
            e = launch_adjoint_step(state, cur, oth, c->force(), c->dims, c->lbm.tau0, cs,
                                    c->lbm.mu, c->storage(), kpart, s);
            if (e != hipSuccess) return hip_fail(e, "adjoint_step");
            std::swap(cur, oth);
        }
        e = hipEventRecord(c->rfree[t % 2], s);
        if (e != hipSuccess) return hip_fail(e, "recompute release");
    }
    e = launch_lam_to_canonical(cur, d_grad_f0, c->dims, s);
    if (e != hipSuccess) return hip_fail(e, "lam_to_canonical");
    if (d_grad_cs) {
        // dK/dC_s = 36 sqrt(2) C_s
        e = launch_sum(kpart, (size_t)nparts, 36.0 * std::sqrt(2.0) * cs, d_grad_cs, s);
        if (e != hipSuccess) return hip_fail(e, "sum");
    }
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_moments(lbmletkf_ctx* ctx, const void* d_f, double* d_out, void* stream) {
    Ctx* c = as_ctx(ctx);
    if (!c || !d_f || !d_out) return fail(LBMLETKF_EINVAL, "NULL argument");
    hipError_t e = launch_moments(d_f, d_out, c->dims, c->storage(), as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "moments");
}

lbmletkf_status lbmletkf_synth_obs(const double* d_y, const double* d_eps, const double* d_sigma,
                                   double* d_yo, int32_t n, void* stream) {
    if (!d_y || !d_eps || !d_sigma || !d_yo) return fail(LBMLETKF_EINVAL, "NULL argument");
    if (n < 0) return fail(LBMLETKF_EINVAL, "n must be >= 0");
    if (n == 0) return LBMLETKF_OK;
    hipError_t e = launch_synth_obs(d_y, d_eps, d_sigma, d_yo, n, as_stream(stream));
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "synth_obs");
}

lbmletkf_status lbmletkf_info(lbmletkf_ctx* ctx, int32_t* max_local_points, int32_t* eig_size,
                              int32_t* route) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    if (max_local_points) *max_local_points = c->lmax;
    if (eig_size) *eig_size = c->n_eig;
    if (route) *route = c->route;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_local_histogram(lbmletkf_ctx* ctx, int32_t* hist, int32_t len) {
    Ctx* c = as_ctx(ctx);
    if (!c || !hist || len < 0) return fail(LBMLETKF_EINVAL, "bad argument");
    for (int k = 0; k < len; ++k) hist[k] = k < (int)c->hist.size() ? c->hist[k] : 0;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_set_profiling(lbmletkf_ctx* ctx, int32_t enable) {
    Ctx* c = as_ctx(ctx);
    if (!c) return fail(LBMLETKF_EINVAL, "ctx is NULL");
    if (enable < 0 || enable > 2) return fail(LBMLETKF_EINVAL, "profiling level must be 0, 1 or 2");
    c->profiling = enable;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_profile_collect(lbmletkf_ctx* ctx, double* ms, int64_t* counts) {
    Ctx* c = as_ctx(ctx);
    if (!c || !ms || !counts) return fail(LBMLETKF_EINVAL, "NULL argument");
    for (int k = 0; k < LBMLETKF_NSTAGES; ++k) {
        ms[k] = 0.0;
        counts[k] = 0;
    }
    lbmletkf_status st = LBMLETKF_OK;
    for (auto& r : c->recs) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess && st == LBMLETKF_OK) st = hip_fail(e, "profile_collect");
        ms[r.stage] += t;
        counts[r.stage] += r.launches;
        c->event_pool.push_back(r.a);
        c->event_pool.push_back(r.b);
    }
    c->recs.clear();
    return st;
}

}  // extern "C"

// ===========================================================================
// Batching form: many independent problems (contexts) per cycle.
// ===========================================================================
namespace {

// Smallest instantiated observation-route size >= n that is a multiple of g.
int coarse_size(int n, int g) {
    int v = obs_size_for(n);
    while (v != 0 && v % g != 0) v = obs_size_for(v + 1);
    return v;
}

struct BatchGroup {
    int route;  // LBMLETKF_ROUTE_ENSEMBLE or LBMLETKF_ROUTE_OBSERVATION
    int n;      // eigenproblem size
    int stream; // 0: the launch stream, k > 0: side stream k - 1
    int4* eig_waves = nullptr;
    int n_eig = 0;
    int2* waves = nullptr;  // apply waves (observation route) or node waves (ensemble route)
    int n_waves = 0;
    int* nodes = nullptr;
    double* gbuf = nullptr;
    int nz_max = 0;
    double cost = 0.0;
};

struct Batch {
    std::vector<Ctx*> ctx;
    std::vector<void*> f;
    int nsteps = 0;
    int storage = 0;
    bool mfma_transform = false;  // every context's setting, taken at create
    lbmletkf_batch_config cfg{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    AnalysisParams* d_params = nullptr;       // [n], f = the bound states
    AnalysisParams* d_params_tune = nullptr;  // [n], f = the ping-pong partners
    LbmTask* d_tasks[3] = {nullptr, nullptr, nullptr};  // even, odd, tuning steps
    double* d_yo = nullptr;
    std::vector<size_t> yo_off;
    char* gbase = nullptr;  // group region
    size_t gcap = 0;
    int* d_queue = nullptr;  // [16 per group] work-queue counters (analysis_queue = 1)
    std::vector<BatchGroup> groups;
    int ntiles = 0;
    int nblocks2 = 0;  // blocks of a batched two-step launch
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {nullptr, nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

Batch* as_batch(lbmletkf_batch* b) { return reinterpret_cast<Batch*>(b); }

struct BatchLayout {
    size_t params, tasks, yo, queue, groups, total, group_bytes;
};

// Work-queue counters of the batched analysis: 16 per group, at most one group
// per (route, eigenproblem size <= 64).
constexpr int kQueueInts = 16 * 2 * 65;

BatchLayout batch_layout(const std::vector<Ctx*>& ctx) {
    BatchLayout L{};
    const size_t n = ctx.size();
    size_t nobs = 0, nodes = 0, gdoubles = 0;
    for (const Ctx* c : ctx) {
        nobs += c->nobs;
        const size_t plane = (size_t)c->dims.nx * c->dims.ny;
        nodes += plane;
        if (c->route == LBMLETKF_ROUTE_OBSERVATION)
            for (const Bucket& b : c->buckets) {
                const int nc = coarse_size(b.n, 8);  // the largest size any granularity gives
                gdoubles += obs_gbuf_doubles(nc, b.count);
            }
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    // [2n]: the bound states' parameters, then the partners' (one copy at create)
    L.params = take(2 * n * sizeof(AnalysisParams));
    L.tasks = take(3 * n * sizeof(LbmTask));
    L.yo = take(nobs * sizeof(double));
    L.queue = take(kQueueInts * sizeof(int));
    // groups: node lists, eigen waves, apply/ensemble waves, G buffers (+ alignment slack
    // for up to 64 groups of four arrays)
    L.group_bytes = nodes * (sizeof(int) + sizeof(int4) + sizeof(int2)) + gdoubles * sizeof(double) +
                    64 * 4 * kAlign;
    L.groups = take(L.group_bytes);
    L.total = off;
    return L;
}

void batch_release(Batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (int k = 0; k < Batch::kSide; ++k) {
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
}

// Forecast tasks for the tile configuration: even steps f -> partner, odd steps
// partner -> f, tuning steps f -> partner (the bound states stay untouched).
lbmletkf_status batch_tasks(Batch* b, hipStream_t s) {
    const int n = (int)b->ctx.size();
    std::vector<LbmTask> t(3 * n);
    int tile0 = 0, block0 = 0;
    for (int k = 0; k < n; ++k) {
        const Ctx* c = b->ctx[k];
        const int M = c->dims.members;
        // a tile row is one block's worth of nodes: 256 threads, M / V per node
        // (V = 2 members per thread for FP32 storage with even M)
        const int V = (c->storage() == kStoreF32Dev && M % 2 == 0) ? 2 : 1;
        const int tile_nodes = b->cfg.tile_rows * (256 / (M / V));
        const int plane = c->dims.nx * c->dims.ny;
        for (int v = 0; v < 3; ++v) {
            LbmTask& x = t[v * n + k];
            x.fin = v == 1 ? c->fbuf() : b->f[k];
            x.fout = v == 1 ? b->f[k] : c->fbuf();
            x.force = c->force();
            x.nx = c->dims.nx;
            x.ny = c->dims.ny;
            x.members = M;
            x.tile_nodes = tile_nodes;
            x.tile0 = tile0;
            x.block0 = block0;
            x.tau0 = c->lbm.tau0;
            x.smag = 18.0 * std::sqrt(2.0) * c->lbm.cs * c->lbm.cs;
            x.mu = c->lbm.mu;
        }
        tile0 += (plane + tile_nodes - 1) / tile_nodes;
        if (two_step_supported(c->dims, c->storage()))
            block0 += two_step_blocks(c->dims, c->storage());
    }
    b->ntiles = tile0;
    b->nblocks2 = block0;
    hipError_t e = hipMemcpyAsync(b->d_tasks[0], t.data(), t.size() * sizeof(LbmTask),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "batch tasks");
}

// Analysis groups for the bucket granularity: one group per (route, size) across problems.
lbmletkf_status batch_groups(Batch* b, hipStream_t s) {
    const int n = (int)b->ctx.size();
    const int g = b->cfg.bucket_granularity;
    struct Range { int k, offset, count; };
    std::vector<std::vector<Range>> obs(65);
    std::vector<std::vector<int>> ens(65);
    for (int k = 0; k < n; ++k) {
        const Ctx* c = b->ctx[k];
        if (c->route == LBMLETKF_ROUTE_OBSERVATION) {
            for (const Bucket& bk : c->buckets)
                if (bk.count > 0) obs[coarse_size(bk.n, g)].push_back({k, bk.offset, bk.count});
        } else {
            ens[c->n_eig].push_back(k);
        }
    }
    b->groups.clear();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return b->gbase + at;
    };
    std::vector<std::vector<int4>> host_eig;
    std::vector<std::vector<int2>> host_waves;
    struct NodeCopy { int* dst; const int* src; size_t count; };
    std::vector<NodeCopy> node_copies;  // issued once the layout is known to fit
    hipError_t e = hipSuccess;
    for (int sz = 0; sz <= 64; ++sz) {
        if (!obs[sz].empty()) {
            BatchGroup grp;
            grp.route = LBMLETKF_ROUTE_OBSERVATION;
            grp.n = sz;
            int total = 0;
            for (const Range& r : obs[sz]) total += r.count;
            grp.nodes = reinterpret_cast<int*>(take((size_t)total * sizeof(int)));
            std::vector<int4> ew;
            std::vector<int2> aw;
            const int segs = obs_segments(sz);
            int base = 0;
            for (const Range& r : obs[sz]) {
                node_copies.push_back({grp.nodes + base, b->ctx[r.k]->nodes() + r.offset,
                                       (size_t)r.count});
                for (int i = 0; i < r.count; i += segs) ew.push_back(make_int4(r.k, base + i, base + r.count, 0));
                for (int i = 0; i < r.count; ++i) aw.push_back(make_int2(r.k, base + i));
                grp.cost += (double)r.count * obs_node_cost(sz);
                base += r.count;
            }
            grp.n_eig = (int)ew.size();
            grp.n_waves = (int)aw.size();
            grp.eig_waves = reinterpret_cast<int4*>(take(ew.size() * sizeof(int4)));
            grp.waves = reinterpret_cast<int2*>(take(aw.size() * sizeof(int2)));
            grp.gbuf = reinterpret_cast<double*>(take(obs_gbuf_doubles(sz, total) * sizeof(double)));
            host_eig.push_back(std::move(ew));
            host_waves.push_back(std::move(aw));
            b->groups.push_back(grp);
        }
        if (!ens[sz].empty()) {
            BatchGroup grp;
            grp.route = LBMLETKF_ROUTE_ENSEMBLE;
            grp.n = sz;
            std::vector<int2> w;
            for (int k : ens[sz]) {
                const Ctx* c = b->ctx[k];
                const int plane = c->dims.nx * c->dims.ny;
                for (int i = 0; i < plane; i += ens_segments(sz)) w.push_back(make_int2(k, i));
                grp.nz_max = std::max(grp.nz_max, c->obs.nvar * c->lmax);
                grp.cost += (double)plane * ens_node_cost(sz);
            }
            grp.n_waves = (int)w.size();
            grp.waves = reinterpret_cast<int2*>(take(w.size() * sizeof(int2)));
            host_eig.emplace_back();
            host_waves.push_back(std::move(w));
            b->groups.push_back(grp);
        }
    }
    if (off > b->gcap) return fail(LBMLETKF_EWORKSPACE, "batch workspace too small for its groups");
    if (16 * b->groups.size() > (size_t)kQueueInts)
        return fail(LBMLETKF_EUNSUPPORTED, "more analysis groups than work-queue counters");
    for (const NodeCopy& nc : node_copies) {
        e = hipMemcpyAsync(nc.dst, nc.src, nc.count * sizeof(int), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "batch node lists");
    }
    for (size_t i = 0; i < b->groups.size() && e == hipSuccess; ++i) {
        BatchGroup& grp = b->groups[i];
        if (!host_eig[i].empty())
            e = hipMemcpyAsync(grp.eig_waves, host_eig[i].data(), host_eig[i].size() * sizeof(int4),
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !host_waves[i].empty())
            e = hipMemcpyAsync(grp.waves, host_waves[i].data(), host_waves[i].size() * sizeof(int2),
                               hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "batch waves");
    // longest processing time first over the launch stream and the side streams,
    // on the measured per-node costs of each route and size (the two routes'
    // kernels differ too much for a common N^3 model: the packed 16-member
    // ensemble route costs 1/44 of a 48-observation node)
    std::vector<int> order(b->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->groups[x].cost > b->groups[y].cost; });
    double load[1 + Batch::kSide] = {0.0, 0.0, 0.0, 0.0};
    for (int i : order) {
        int best = 0;
        for (int k = 1; k <= Batch::kSide; ++k)
            if (load[k] < load[best]) best = k;
        b->groups[i].stream = best;
        load[best] += b->groups[i].cost;
    }
    std::vector<BatchGroup> sorted;
    for (int i : order) sorted.push_back(b->groups[i]);
    b->groups.swap(sorted);
    return LBMLETKF_OK;
}

// The analyses of all problems (statistics already done), forked over the streams.
hipError_t batch_analysis(Batch* b, const AnalysisParams* params, hipStream_t s) {
    bool used[Batch::kSide] = {false, false, false};
    for (const BatchGroup& grp : b->groups)
        if (grp.stream > 0) used[grp.stream - 1] = true;
    const bool queue = b->cfg.analysis_queue == 1;
    hipError_t e = queue ? launch_zero_ints(b->d_queue, 16 * (int)b->groups.size(), s) : hipSuccess;
    if (e == hipSuccess) e = hipEventRecord(b->fork, s);
    for (int k = 0; k < Batch::kSide && e == hipSuccess; ++k)
        if (used[k]) e = hipStreamWaitEvent(b->side[k], b->fork, 0);
    for (const BatchGroup& grp : b->groups) {
        if (e != hipSuccess) break;
        hipStream_t sk = grp.stream == 0 ? s : b->side[grp.stream - 1];
        if (grp.route == LBMLETKF_ROUTE_OBSERVATION && queue)
            e = launch_analysis_obs_batch_queue(params, grp.eig_waves, grp.n_eig, grp.waves,
                                                grp.n_waves, grp.nodes, grp.n, grp.gbuf,
                                                b->storage, b->mfma_transform,
                                                b->d_queue + 16 * (&grp - b->groups.data()), sk);
        else if (grp.route == LBMLETKF_ROUTE_OBSERVATION)
            e = launch_analysis_obs_batch(params, grp.eig_waves, grp.n_eig, grp.waves, grp.n_waves,
                                          grp.nodes, grp.n, grp.gbuf, b->storage,
                                          b->mfma_transform, sk);
        else
            e = launch_analysis_ens_batch(params, grp.waves, grp.n_waves, grp.n, grp.nz_max,
                                          b->storage, sk);
    }
    for (int k = 0; k < Batch::kSide && e == hipSuccess; ++k) {
        if (!used[k]) continue;
        e = hipEventRecord(b->join[k], b->side[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[k], 0);
    }
    return e;
}

// Observation operator and statistics of every problem (inputs: the bound states
// or, for tuning, their partners).
hipError_t batch_observe(Batch* b, bool partners, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < b->ctx.size() && e == hipSuccess; ++k) {
        Ctx* c = b->ctx[k];
        const void* f = partners ? c->fbuf() : b->f[k];
        e = launch_observe(f, c->pts(), c->obs.n_points, c->obs.nvar, c->yf(), c->dims,
                           b->storage, s);
        if (e == hipSuccess)
            e = launch_obs_stats(c->yf(), b->d_yo + b->yo_off[k], c->nobs, c->dims.members,
                                 c->ybar(), c->dY(), c->dvec(), c->K(), b->storage, s);
    }
    return e;
}

// Blocks of the batched forecast launch: the configured persistent count, or
// one block per tile (forecast_blocks = 0).
int forecast_grid(const Batch* b) {
    return b->cfg.forecast_blocks > 0 ? b->cfg.forecast_blocks : std::max(b->ntiles, 1);
}

// Whether every problem of the batch can take two steps per launch.
bool batch_two_step_ok(const Batch* b) {
    for (const Ctx* c : b->ctx)
        if (!two_step_supported(c->dims, c->storage())) return false;
    return true;
}

// The forecast of every problem: nsteps steps in launches of one or two steps
// (config), alternating between the bound states and their partners; an odd
// number of launches leaves the result in the partners, which are copied back.
hipError_t batch_forecast(Batch* b, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int n = (int)b->ctx.size();
    const bool two = b->cfg.steps_per_launch == 2;
    int launches = 0;
    for (int step = 0; step < b->nsteps && e == hipSuccess; ++launches) {
        const LbmTask* tasks = b->d_tasks[launches & 1];
        if (two && b->nsteps - step >= 2) {
            e = launch_stream_collide2_batch(tasks, n, b->nblocks2, b->storage, s);
            step += 2;
        } else {
            e = launch_stream_collide_batch(tasks, n, b->ntiles, forecast_grid(b), b->storage, s);
            step += 1;
        }
    }
    if (launches & 1)
        for (int k = 0; k < n && e == hipSuccess; ++k)
            e = hipMemcpyAsync(b->f[k], b->ctx[k]->fbuf(), b->ctx[k]->state_bytes(),
                               hipMemcpyDeviceToDevice, s);
    return e;
}

// One whole cycle of every problem on stream s.
hipError_t batch_issue_cycle(Batch* b, hipStream_t s) {
    hipError_t e = batch_forecast(b, s);
    if (e == hipSuccess) e = batch_observe(b, false, s);
    if (e == hipSuccess) e = batch_analysis(b, b->d_params, s);
    return e;
}

lbmletkf_status batch_capture(Batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (!b->cfg.use_graph) return LBMLETKF_OK;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "batch capture");
    hipError_t e2 = batch_issue_cycle(b, b->cap);
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (e2 != hipSuccess) return hip_fail(e2, "batch capture launches");
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "batch graph");
}

lbmletkf_status batch_check_config(const lbmletkf_batch_config* cfg) {
    if (cfg->forecast_blocks < 0 || cfg->forecast_blocks > (1 << 20))
        return fail(LBMLETKF_EINVAL, "forecast_blocks must be in 0..2^20");
    if (cfg->tile_rows < 1 || cfg->tile_rows > 64)
        return fail(LBMLETKF_EINVAL, "tile_rows must be in 1..64");
    if (cfg->bucket_granularity != 2 && cfg->bucket_granularity != 4 &&
        cfg->bucket_granularity != 8)
        return fail(LBMLETKF_EINVAL, "bucket_granularity must be 2, 4 or 8");
    if (cfg->steps_per_launch != 1 && cfg->steps_per_launch != 2)
        return fail(LBMLETKF_EINVAL, "steps_per_launch must be 1 or 2");
    if (cfg->analysis_queue != 0 && cfg->analysis_queue != 1)
        return fail(LBMLETKF_EINVAL, "analysis_queue must be 0 or 1");
    return LBMLETKF_OK;
}

lbmletkf_status batch_apply_config(Batch* b, const lbmletkf_batch_config* cfg, hipStream_t s) {
    lbmletkf_status st = batch_check_config(cfg);
    if (st) return st;
    if (cfg->steps_per_launch == 2 && !batch_two_step_ok(b))
        return fail(LBMLETKF_EUNSUPPORTED, "two steps per launch need 16 | members in every problem");
    b->cfg = *cfg;
    if ((st = batch_tasks(b, s))) return st;
    if ((st = batch_groups(b, s))) return st;
    return batch_capture(b);
}

}  // namespace

extern "C" {

lbmletkf_status lbmletkf_batch_workspace_bytes(lbmletkf_ctx* const* ctxs, int32_t n, size_t* bytes) {
    if (!ctxs || n < 1 || !bytes) return fail(LBMLETKF_EINVAL, "need n >= 1 contexts and bytes");
    std::vector<Ctx*> v;
    for (int k = 0; k < n; ++k) {
        if (!ctxs[k]) return fail(LBMLETKF_EINVAL, "NULL context");
        v.push_back(as_ctx(ctxs[k]));
    }
    *bytes = batch_layout(v).total;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_batch_create(lbmletkf_ctx* const* ctxs, void* const* d_f, int32_t n,
                                      int32_t nsteps, const lbmletkf_batch_config* cfg,
                                      void* d_workspace, size_t bytes, void* stream,
                                      lbmletkf_batch** batch_out) {
    if (!ctxs || !d_f || n < 1 || !batch_out) return fail(LBMLETKF_EINVAL, "NULL argument");
    *batch_out = nullptr;
    if (nsteps < 1) return fail(LBMLETKF_EINVAL, "nsteps must be >= 1");
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign))
        return fail(LBMLETKF_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    lbmletkf_batch_config c0{0, 4, 2, 1, 1, 0};
    const lbmletkf_batch_config* use = cfg ? cfg : &c0;
    lbmletkf_status st = batch_check_config(use);
    if (st) return st;
    std::vector<Ctx*> v;
    for (int k = 0; k < n; ++k) {
        if (!ctxs[k] || !d_f[k]) return fail(LBMLETKF_EINVAL, "NULL context or state");
        Ctx* c = as_ctx(ctxs[k]);
        if (c->dims.members < 2) return fail(LBMLETKF_EINVAL, "analysis needs >= 2 members");
        if (256 % c->dims.members != 0)
            return fail(LBMLETKF_EUNSUPPORTED, "batched members must divide 256");
        if (k > 0 && c->storage() != v[0]->storage())
            return fail(LBMLETKF_EUNSUPPORTED, "every problem of a batch needs the same storage");
        if (k > 0 && c->mfma_transform != v[0]->mfma_transform)
            return fail(LBMLETKF_EUNSUPPORTED,
                        "every problem of a batch needs the same matrix-core transform setting");
        for (void* g : std::vector<void*>(d_f, d_f + k))
            if (g == d_f[k]) return fail(LBMLETKF_EINVAL, "two problems share a state buffer");
        v.push_back(c);
    }
    const BatchLayout L = batch_layout(v);
    if (bytes < L.total) return fail(LBMLETKF_EWORKSPACE, "batch workspace too small");
    Batch* b = new Batch();
    b->ctx = v;
    b->f.assign(d_f, d_f + n);
    b->nsteps = nsteps;
    b->storage = v[0]->storage();
    b->mfma_transform = v[0]->mfma_transform;
    b->ws = reinterpret_cast<char*>(d_workspace);
    b->ws_bytes = bytes;
    b->d_params = reinterpret_cast<AnalysisParams*>(b->ws + L.params);
    b->d_params_tune = b->d_params + n;
    b->d_tasks[0] = reinterpret_cast<LbmTask*>(b->ws + L.tasks);
    b->d_tasks[1] = b->d_tasks[0] + n;
    b->d_tasks[2] = b->d_tasks[0] + 2 * n;
    b->d_yo = reinterpret_cast<double*>(b->ws + L.yo);
    b->d_queue = reinterpret_cast<int*>(b->ws + L.queue);
    b->gbase = b->ws + L.groups;
    b->gcap = L.group_bytes;
    size_t yo = 0;
    for (Ctx* c : v) {
        b->yo_off.push_back(yo);
        yo += c->nobs;
    }
    hipStream_t s = as_stream(stream);
    std::vector<AnalysisParams> p(2 * n);
    for (int k = 0; k < n; ++k) {
        p[k] = make_params(v[k], d_f[k]);
        p[n + k] = make_params(v[k], v[k]->fbuf());
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int k = 0; k < Batch::kSide && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_params, p.data(), 2 * n * sizeof(AnalysisParams),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        batch_release(b);
        delete b;
        return hip_fail(e, "lbmletkf_batch_create");
    }
    lbmletkf_batch_config first = *use;
    if (!cfg && batch_two_step_ok(b)) first.steps_per_launch = 2;  // default: two where possible
    if ((st = batch_apply_config(b, &first, s))) {
        batch_release(b);
        delete b;
        return st;
    }
    *batch_out = reinterpret_cast<lbmletkf_batch*>(b);
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_batch_destroy(lbmletkf_batch* batch) {
    Batch* b = as_batch(batch);
    if (!b) return fail(LBMLETKF_EINVAL, "batch is NULL");
    batch_release(b);
    delete b;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_batch_run_cycle(lbmletkf_batch* batch, const double* const* d_yo, void* stream) {
    Batch* b = as_batch(batch);
    if (!b || !d_yo) return fail(LBMLETKF_EINVAL, "NULL argument");
    hipStream_t s = as_stream(stream);
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < b->ctx.size() && e == hipSuccess; ++k) {
        if (!d_yo[k]) return fail(LBMLETKF_EINVAL, "NULL observation vector");
        e = hipMemcpyAsync(b->d_yo + b->yo_off[k], d_yo[k], b->ctx[k]->nobs * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = b->exec ? hipGraphLaunch(b->exec, s) : batch_issue_cycle(b, s);
    return e == hipSuccess ? LBMLETKF_OK : hip_fail(e, "batch cycle");
}

lbmletkf_status lbmletkf_batch_get_config(lbmletkf_batch* batch, lbmletkf_batch_config* cfg) {
    Batch* b = as_batch(batch);
    if (!b || !cfg) return fail(LBMLETKF_EINVAL, "NULL argument");
    *cfg = b->cfg;
    return LBMLETKF_OK;
}

lbmletkf_status lbmletkf_batch_set_config(lbmletkf_batch* batch, const lbmletkf_batch_config* cfg,
                                          void* stream) {
    Batch* b = as_batch(batch);
    if (!b || !cfg) return fail(LBMLETKF_EINVAL, "NULL argument");
    return batch_apply_config(b, cfg, as_stream(stream));
}

lbmletkf_status lbmletkf_batch_tune(lbmletkf_batch* batch, int32_t reps, lbmletkf_batch_config* best,
                                    double* forecast_ms, double* analysis_ms, void* stream) {
    Batch* b = as_batch(batch);
    if (!b || reps < 1) return fail(LBMLETKF_EINVAL, "need a batch and reps >= 1");
    hipStream_t s = as_stream(stream);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    auto timed = [&](auto&& body, double* ms) -> hipError_t {
        hipError_t r = body();  // warm-up (and first-use setup)
        if (r == hipSuccess) r = hipEventRecord(t0, s);
        for (int i = 0; i < reps && r == hipSuccess; ++i) r = body();
        if (r == hipSuccess) r = hipEventRecord(t1, s);
        if (r == hipSuccess) r = hipEventSynchronize(t1);
        float t = 0.0f;
        if (r == hipSuccess) r = hipEventElapsedTime(&t, t0, t1);
        *ms = t / reps;
        return r;
    };
    lbmletkf_batch_config cur = b->cfg;
    cur.use_graph = 0;
    lbmletkf_batch_config best_cfg = cur;
    double best_f = 1e30, best_a = 1e30;
    lbmletkf_status st = LBMLETKF_OK;
    // forecast: persistent blocks (0: one block per tile) x tile rows, stepping the
    // bound states into their partners (the bound states are not modified)
    const int blocks[] = {256, 512, 1024, 2048, 0};
    const int rows[] = {1, 2, 4, 8};
    for (int bl : blocks) {
        for (int tr : rows) {
            if (e != hipSuccess || st) break;
            cur.forecast_blocks = bl;
            cur.tile_rows = tr;
            b->cfg = cur;
            if ((st = batch_tasks(b, s))) break;
            double ms = 0.0;
            const int grid = forecast_grid(b);
            e = timed([&]() {
                return launch_stream_collide_batch(b->d_tasks[2], (int)b->ctx.size(), b->ntiles,
                                                   grid, b->storage, s);
            }, &ms);
            if (e == hipSuccess && ms < best_f) {
                best_f = ms;
                best_cfg.forecast_blocks = bl;
                best_cfg.tile_rows = tr;
                best_cfg.steps_per_launch = 1;
            }
        }
    }
    // two steps per launch over the concatenated (problem, tile, member group)
    // blocks, priced per step
    if (e == hipSuccess && !st && batch_two_step_ok(b)) {
        double ms = 0.0;
        e = timed([&]() {
            return launch_stream_collide2_batch(b->d_tasks[2], (int)b->ctx.size(), b->nblocks2,
                                                b->storage, s);
        }, &ms);
        if (e == hipSuccess && ms / 2 < best_f) {
            best_f = ms / 2;
            best_cfg.steps_per_launch = 2;
        }
    }
    // analysis: bucket granularity, on copies of the states in the partner buffers
    for (size_t k = 0; k < b->ctx.size() && e == hipSuccess && !st; ++k)
        e = hipMemcpyAsync(b->ctx[k]->fbuf(), b->f[k], b->ctx[k]->state_bytes(),
                           hipMemcpyDeviceToDevice, s);
    // (the work-queue form keeps the batch's current setting: it measured about
    // four times slower than one launch per group, so timing it is wasted here)
    const int grans[] = {2, 4, 8};
    for (int g : grans) {
        if (e != hipSuccess || st) break;
        cur = best_cfg;
        cur.bucket_granularity = g;
        b->cfg = cur;
        if ((st = batch_groups(b, s))) break;
        double ms = 0.0;
        e = batch_observe(b, true, s);
        if (e == hipSuccess) e = timed([&]() { return batch_analysis(b, b->d_params_tune, s); }, &ms);
        if (e == hipSuccess && ms < best_a) {
            best_a = ms;
            best_cfg.bucket_granularity = g;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e, "batch tune");
    if (st) return st;
    best_cfg.use_graph = 1;
    if ((st = batch_apply_config(b, &best_cfg, s))) return st;
    if (best) *best = best_cfg;
    if (forecast_ms) *forecast_ms = best_f;
    if (analysis_ms) *analysis_ms = best_a;
    return LBMLETKF_OK;
}

}  // extern "C"
