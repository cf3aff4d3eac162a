// Host driver of the C ABI declared in include/rk.h.
//
// The context owns no device allocation: every device buffer is carved out of
// the caller's workspace.  All device work is enqueued on the context stream;
// the only device-to-host transfers in a time step are the Arnoldi scalars of
// each FGMRES iteration (one small copy and one stream synchronisation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "rk_internal.h"

using namespace rk;

namespace rk {
hipError_t launch_op_k1(const OpLaunch&);
hipError_t launch_op_k2(const OpLaunch&);
hipError_t launch_op_k3(const OpLaunch&);
hipError_t launch_op_k4(const OpLaunch&);
hipError_t launch_op_k5(const OpLaunch&);
hipError_t launch_op_k6(const OpLaunch&);

hipError_t launch_op(const OpLaunch& L) {
    switch (L.k) {
        case 1: return launch_op_k1(L);
        case 2: return launch_op_k2(L);
        case 3: return launch_op_k3(L);
        case 4: return launch_op_k4(L);
        case 5: return launch_op_k5(L);
        case 6: return launch_op_k6(L);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_op_list_k1(const OpLaunch*, int, hipStream_t);
hipError_t launch_op_list_k2(const OpLaunch*, int, hipStream_t);
hipError_t launch_op_list_k3(const OpLaunch*, int, hipStream_t);
hipError_t launch_op_list_k4(const OpLaunch*, int, hipStream_t);
hipError_t launch_op_list_k5(const OpLaunch*, int, hipStream_t);
hipError_t launch_op_list_k6(const OpLaunch*, int, hipStream_t);

hipError_t launch_op_list(const OpLaunch* L, int count, hipStream_t st) {
    if (count < 1) return hipErrorInvalidValue;
    switch (L[0].k) {
        case 1: return launch_op_list_k1(L, count, st);
        case 2: return launch_op_list_k2(L, count, st);
        case 3: return launch_op_list_k3(L, count, st);
        case 4: return launch_op_list_k4(L, count, st);
        case 5: return launch_op_list_k5(L, count, st);
        case 6: return launch_op_list_k6(L, count, st);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace rk

namespace {

constexpr int kRedBlocks = 2048;     // blocks of the reduction kernels
// rk_apply_operator_batch: problems of at least this many stage-DoFs per
// launch fill the GPU alone and take their own tuned launch
constexpr double kOpListAlone = 8.0 * (1 << 20);
// Split V-cycles only from this many fine-level stage-DoFs per V-cycle on:
// smaller V-cycles are latency-bound on every level, and two branches of
// them gain nothing.
constexpr long long kSplitMin = 1ll << 23;
// slots (x 81 doubles) of the device Q x Q mixing data
constexpr int kMixSinv = 0, kMixS = 81, kMixRhs = 162, kMixAinvS = 243, kMixAinv = 324, kMixA = 405;
// direct diagonalisation: Lam_r, PRESB input and output mixes, Lam_r times the output mix
constexpr int kMixCLam = 486, kMixPin = 567, kMixPout = 648, kMixLamPout = 729, kMixSlots = 10;
constexpr size_t kAlign = 256;

enum Form { F_CALA = 0, F_STAGE = 1, F_BLOCKS = 2, F_K = 3, F_M = 4, F_CBLK = 5, F_NFORMS = 6 };

// Mixing coefficients of one operator form (cell size folded in).
struct Coeffs {
    double alpha[RK_MAX_Q] = {}, beta[RK_MAX_Q] = {};
    bool pair = false;      // two inputs: mass-term input, stiffness-term input
    int premix = 0;         // pair forms: 1 = mass input is (A^-1 (x) I) u, 2 = stiffness input is
                            // (A (x) I) u, 3 = mass input is (Lam_r (x) I) u
};

struct Level {
    int n = 0, N = 0;
    long long N3 = 0;
    double h = 0.0;
    void* b = nullptr;      // [Q][N3], preconditioner dtype
    void* x = nullptr;
    void* y = nullptr;
    Coeffs blk;             // block operators lam_i M + tau K on this level
    double eig_max = 1.0;
    int cz = 0;             // tuned z-chunk of the diagonal-mix operator (0: heuristic),
    int ts = 0;             // and its tile shape, for the V-cycle epilogues
    int cz_st = 0;          // the same for the plain (store) epilogue
    int ts_st = 0;
    // multigrid on the deformed mesh: per-point geometry, Jacobi diagonals of
    // M and K, and an operator output temp ([Q][N3]), preconditioner dtype
    void* geo = nullptr;
    void* dMv = nullptr;
    void* dKv = nullptr;
    void* t = nullptr;
};

struct Event {
    hipEvent_t a, b;
    int comp;
};

struct Carver {
    char* base;
    size_t off = 0;
    size_t cap;
    void* take(size_t bytes) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        void* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

size_t dsize(int dtype) { return dtype == RK_FP64 ? 8 : 4; }

std::string g_create_error;

}  // namespace

struct rk_ctx {
    int n = 0, k = 0, Q = 0, N = 0;
    long long N3 = 0;
    double tau = 0.0, h = 0.0;
    double length = 1.0;           // edge of the cube; h = length / n
    rk_options opt{};
    std::vector<double> eig_user;
    Tableau tab{};
    Element1D el{};
    hipStream_t stream = nullptr;
    int device = 0;                // HIP device current at create
    // The fine-level V-cycle (F.b -> F.x, fixed buffers) is captured once into
    // a HIP graph on a private stream and replayed on `stream`: the coarse
    // levels are tens of small launches whose dispatch cost the graph cuts.
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t vc_exec = nullptr;
    int vc_graph = 0;              // 0 not tried, 1 captured, -1 eager only
    // Split V-cycles (opt.vc_streams groups of stage blocks): group g > 0
    // runs on aux_stream[g], forked from and joined back into `stream` by
    // events, so that the latency-bound coarse levels of one group overlap the
    // fine levels of another.  Created on first use.
    hipStream_t aux_stream[RK_MAX_Q] = {};
    hipEvent_t ev_fork = nullptr, ev_join[RK_MAX_Q] = {};
    int pc = RK_FP64;              // preconditioner dtype
    bool cplx = false;             // direct diagonalisation with PRESB
    bool deformed = false;         // Krylov operator and K y_n on the deformed mesh
    bool dmg = false;              // V-cycles on the deformed levels
    void* geo = nullptr;           // its per-point geometry (fp64)
    int ng = 1;                    // independent Krylov systems (complex: the nb blocks)
    Segs seg;                      // their segments of the Krylov vectors
    SlotIdx slot_group;            // slot -> group
    int nscal = 0;                 // per-group stride of scal / scal2 / ycoef
    std::vector<Level> lv;
    Coeffs form[F_NFORMS];         // fine-level operator coefficients
    Coeffs presb_m;                // PRESB coupling: Im(lam_j) M on slots nb + j
    int cz_pair = 0;               // tuned z-chunk of the fine-level fp64 pair operator
    // The coarse end of the V-cycle from level tail_level down runs in one
    // launch (-1: none); its per-stage scratch holds 4 N^3 of that level.
    int tail_level = -1;
    void* tail = nullptr;
    size_t tail_stage = 0;
    void* tmp = nullptr;           // restriction intermediate, [Q][tmp_stage]
    size_t tmp_stage = 0;          // its per-stage size: the largest N_l N_(l+1)^2
    long long ld = 0;              // stride of the Krylov vectors (Q N3 padded to 256 bytes)
    double* V = nullptr;           // (restart+1) x ld
    double* Z = nullptr;           // restart x ld
    double* w = nullptr;           // Q N3
    double* kv = nullptr;          // Q N3
    double* rhs = nullptr;         // Q N3
    double* Ky = nullptr;          // N3
    double* part = nullptr;        // groups x kRedBlocks x nscal
    double* scal = nullptr;        // groups x nscal device scalars
    double* scal2 = nullptr;       // groups x nscal
    double* ycoef = nullptr;       // groups x nscal
    double* sig = nullptr;         // (restart + 16) x kSigStride: 1 / ||Vhat_i|| per group
    double* mix = nullptr;         // kMixSlots x 81: the Q x Q mixing matrices
    void* mbuf = nullptr;          // Q N3 (fp64-sized): mixed input of the pair operators
    std::vector<double> host_scal;
    std::vector<Event> events;
    std::vector<Event> event_pool;
    size_t pool_used = 0;
    std::string err;
};

namespace {

int fail(rk_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, RK_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

std::vector<int> level_cells(int n) {
    std::vector<int> out{n};
    while (out.back() % 2 == 0 && (int)out.size() < RK_MAX_LEVELS) out.push_back(out.back() / 2);
    return out;
}

bool valid_options(const rk_options& o, std::string& msg) {
    if (o.precision != RK_PREC_FP64 && o.precision != RK_PREC_MIXED) { msg = "bad precision"; return false; }
    if (o.mode != RK_BATCHED && o.mode != RK_PER_STAGE) { msg = "bad mode"; return false; }
    if (!(o.rtol > 0.0) || o.max_iter < 1 || o.restart < 1 || o.restart > 256) { msg = "bad FGMRES settings"; return false; }
    if (o.cheb_degree < 1 || o.coarse_cheb_degree < 1 || o.cheb_degree > 64 || o.coarse_cheb_degree > 64) {
        msg = "bad Chebyshev degree"; return false;
    }
    if (!(o.cheb_range > 1.0) || !(o.eig_safety > 0.0) || o.eig_iterations < 1) { msg = "bad Chebyshev interval settings"; return false; }
    if (o.method != RK_METHOD_CROUT && o.method != RK_METHOD_COMPLEX) { msg = "bad method"; return false; }
    if (o.autotune != 0 && o.autotune != 1) { msg = "bad autotune flag"; return false; }
    if (o.deform_mg != 0 && o.deform_mg != 1) { msg = "bad deform_mg flag"; return false; }
    if (o.vc_streams < 1 || o.vc_streams > RK_MAX_Q) { msg = "vc_streams out of range"; return false; }
    if (o.z_chunk < 0 || o.z_chunk > 64) { msg = "z_chunk out of range (0..64)"; return false; }
    if (o.tile_shape != 0 && o.tile_shape != 1) { msg = "tile_shape must be 0 or 1"; return false; }
    if (o.tail_nodes < 0) { msg = "tail_nodes must be >= 0"; return false; }
    if (!(std::fabs(o.deform) <= RK_MAX_DEFORM)) { msg = "|deform| must be <= RK_MAX_DEFORM"; return false; }
    return true;
}

// Coefficients of an operator form on a grid with cell size h:
//   CALA:   v_s = h^3 Mref (sum_j Ainv_sj u_j) + tau h Kref u_s    (eq. irk:A)
//   STAGE:  v_s = h^3 Mref u_s + tau h Kref (sum_j A_sj u_j)       (stage system)
// (the Q x Q mix of the dense forms is applied to the input by a streaming
// kernel, then the pair operator runs on (mixed input, plain input))
//   BLOCKS: v_s = lam_s h^3 Mref u_s + tau h Kref u_s              (eq. irk:P blocks)
//   K, M:   one vector.
//   CBLK:   v_s = h^3 Mref (sum_j Lam_r,sj u_j) + tau h Kref u_s   (Sec. 6 blocks)
// The multigrid blocks of a level are lam_i M + tau K (eq. irk:P), or for the
// complex method the PRESB matrices H = (Re lam + Im lam) M + tau K per slot.
Coeffs make_coeffs(const rk_ctx& c, double h, int form) {
    const int Q = c.Q;
    Coeffs r;
    const double h3 = h * h * h;
    for (int s = 0; s < RK_MAX_Q; ++s) {
        if (form == F_BLOCKS && s < Q) {
            r.alpha[s] = (c.cplx ? c.tab.hshift[s] : c.tab.lam[s]) * h3;
            r.beta[s] = c.tau * h;
        }
        if (form == F_K) { r.alpha[s] = 0.0; r.beta[s] = h; }
        if (form == F_M) { r.alpha[s] = h3; r.beta[s] = 0.0; }
    }
    if (form == F_CALA || form == F_STAGE || form == F_CBLK) {
        r.pair = true;
        r.premix = form == F_CALA ? 1 : form == F_STAGE ? 2 : 3;
        for (int q = 0; q < Q; ++q) { r.alpha[q] = h3; r.beta[q] = c.tau * h; }
    }
    return r;
}

StageScal to_stage_scal(const Coeffs& cf) {
    StageScal s;
    for (int i = 0; i < RK_MAX_Q; ++i) { s.alpha[i] = cf.alpha[i]; s.beta[i] = cf.beta[i]; }
    return s;
}

// Carve the workspace (base == nullptr: size query).
size_t carve(rk_ctx& c, char* base) {
    Carver cv{base, 0, 0};
    const int Q = c.Q, k = c.k;
    const size_t pcs = dsize(c.pc);
    for (auto& L : c.lv) {
        L.b = cv.take(pcs * Q * L.N3);
        L.x = cv.take(pcs * Q * L.N3);
        L.y = cv.take(pcs * Q * L.N3);
        if (c.dmg) {
            L.geo = cv.take(pcs * deformed_geometry_elems(L.n, k));
            L.dMv = cv.take(pcs * L.N3);
            L.dKv = cv.take(pcs * L.N3);
            L.t = cv.take(pcs * Q * L.N3);
        }
    }
    // restriction intermediate: x-y restricted fine planes of the finest pair
    size_t tmp = 1;
    for (size_t l = 0; l + 1 < c.lv.size(); ++l)
        tmp = std::max(tmp, (size_t)c.lv[l].N * c.lv[l + 1].N * c.lv[l + 1].N);
    c.tmp_stage = tmp;
    c.tmp = cv.take(pcs * Q * tmp);
    if (c.tail_level >= 0) {
        c.tail_stage = 4 * (size_t)c.lv[c.tail_level].N3;
        c.tail = cv.take(pcs * Q * c.tail_stage);
    }
    const long long qn = (long long)Q * c.N3;
    const int m = c.opt.restart;
    // Krylov vectors are qn long, stored at a stride padded to 256 bytes
    c.ld = (qn + 31) / 32 * 32;
    c.V = (double*)cv.take(8 * (size_t)(m + 1) * c.ld);
    c.Z = (double*)cv.take(8 * (size_t)m * c.ld);
    c.w = (double*)cv.take(8 * qn);
    c.kv = (double*)cv.take(8 * qn);
    c.rhs = (double*)cv.take(8 * qn);
    c.Ky = (double*)cv.take(8 * c.N3);
    const size_t nscal = std::max(m + 16, 3 * RK_MAX_Q + 1);
    const size_t ngmax = (size_t)(Q + 1) / 2;
    c.nscal = (int)nscal;
    c.part = (double*)cv.take(8 * (size_t)kRedBlocks * nscal * ngmax);
    c.scal = (double*)cv.take(8 * nscal * ngmax);
    c.scal2 = (double*)cv.take(8 * nscal * ngmax);
    c.ycoef = (double*)cv.take(8 * nscal * ngmax);
    c.sig = (double*)cv.take(8 * (size_t)(m + 16) * kSigStride);
    c.mix = (double*)cv.take(8 * kMixSlots * 81);
    c.mbuf = cv.take(8 * (size_t)qn);
    if (c.deformed) c.geo = cv.take(8 * deformed_geometry_elems(c.n, c.k));
    return cv.off + kAlign;
}

int setup_sizes(rk_ctx& c, const rk_mesh* mesh, int degree, int Q, const rk_options* opt) {
    if (!mesh || mesh->n_cells < 1 || degree < 1 || degree > RK_MAX_DEGREE || Q < 1 || Q > RK_MAX_Q)
        return fail(nullptr, RK_EINVAL, "mesh, degree (1..6) or Q (1..9) out of range");
    if (!(mesh->length > 0.0) || !std::isfinite(mesh->length))
        return fail(nullptr, RK_EINVAL, "mesh length must be finite and > 0");
    // launch grids put (stage, z-plane) pairs in one grid dimension (<= 65535)
    // and operator kernels address a node plane with 32-bit byte offsets
    if ((long long)mesh->n_cells * degree + 1 > std::min(65535 / Q, 16384))
        return fail(nullptr, RK_EINVAL, "grid too large: need (n_cells*degree + 1) <= 16384 and "
                                        "(n_cells*degree + 1) * Q <= 65535");
    if (opt) c.opt = *opt;
    else rk_default_options(&c.opt);
    std::string msg;
    if (!valid_options(c.opt, msg)) return fail(nullptr, RK_EINVAL, msg);
    c.n = mesh->n_cells;
    c.k = degree;
    c.Q = Q;
    c.N = c.n * c.k + 1;
    c.N3 = (long long)c.N * c.N * c.N;
    c.length = mesh->length;
    c.h = c.length / c.n;
    c.pc = c.opt.precision == RK_PREC_MIXED ? RK_FP32 : RK_FP64;
    c.cplx = c.opt.method == RK_METHOD_COMPLEX;
    c.deformed = c.opt.deform != 0.0;
    c.dmg = c.deformed && c.opt.deform_mg == 1;
    if (c.deformed && c.length != 1.0)
        return fail(nullptr, RK_EINVAL, "deformed meshes are defined on the unit cube: mesh length must be 1");
    c.lv.clear();
    for (int m : level_cells(c.n)) {
        Level L;
        L.n = m;
        L.N = m * c.k + 1;
        L.N3 = (long long)L.N * L.N * L.N;
        L.h = c.length / m;
        c.lv.push_back(L);
    }
    // the one-launch coarse end: affine-mesh levels of at most tail_nodes
    // nodes, if the tail kernel can take all of them
    c.tail_level = -1;
    if (!c.dmg && c.opt.tail_nodes > 0)
        for (size_t l = 0; l < c.lv.size(); ++l)
            if (c.lv[l].N3 <= c.opt.tail_nodes) {
                if ((int)(c.lv.size() - l) <= kTailMaxLevels) c.tail_level = (int)l;
                break;
            }
    return RK_OK;
}

// ---------------------------------------------------------------------------
// Component timing with events (only when opt.timing is set).
// ---------------------------------------------------------------------------
enum Comp { C_RHS = 0, C_VMULT, C_BASIS, C_BLOCKS, C_REST, C_N };

struct Timer {
    rk_ctx* c;
    int comp;
    Event* ev = nullptr;
    Timer(rk_ctx* ctx, int cp) : c(ctx), comp(cp) {
        if (!c->opt.timing) return;
        if (c->pool_used == c->event_pool.size()) {
            Event e{};
            (void)hipEventCreate(&e.a);
            (void)hipEventCreate(&e.b);
            c->event_pool.push_back(e);
        }
        ev = &c->event_pool[c->pool_used++];
        ev->comp = comp;
        (void)hipEventRecord(ev->a, c->stream);
    }
    ~Timer() {
        if (ev) (void)hipEventRecord(ev->b, c->stream);
    }
};

// ---------------------------------------------------------------------------
// Operators and the V-cycle.
// ---------------------------------------------------------------------------
// One operator launch.  For pair coefficients u is the mass-term input and
// u2 the stiffness-term input.
OpLaunch op_launch(const rk_ctx* c, int k, int dtype, int epi, const Coeffs& cf, const void* u, void* v,
                   const void* b, const void* xo, int n, int s0, int ns, double ca, double cb,
                   const void* u2 = nullptr, int xo_from_b = 0, double c0 = 0.0) {
    OpLaunch L;
    L.xo_from_b = xo_from_b; L.c0 = c0;
    L.k = k; L.dtype = dtype; L.mix = cf.pair ? MIX_PAIR : MIX_DIAG; L.epi = epi;
    L.u = u; L.u2 = u2; L.v = v; L.b = b; L.xo = xo;
    for (int i = 0; i < RK_MAX_Q; ++i) { L.alpha[i] = cf.alpha[i]; L.beta[i] = cf.beta[i]; }
    const long long N = (long long)n * k + 1;
    L.stride = N * N * N;
    L.n = n; L.s0 = s0; L.nstage = ns; L.ca = ca; L.cb = cb;
    L.stream = c->stream;
    // tuned z-chunk: pair operators of the fine level in fp64, diagonal-mix
    // operators of every level in the preconditioner precision
    if (c->opt.z_chunk > 0) {
        L.cz = c->opt.z_chunk;
        // the fixed tile shape applies to the fp32 diagonal-mix kernels
        if (!cf.pair && dtype == RK_FP32) L.ts = c->opt.tile_shape;
    } else if (cf.pair) {
        if (n == c->n && dtype == RK_FP64) L.cz = c->cz_pair;
    } else if (dtype == c->pc) {
        for (const auto& lv : c->lv)
            if (lv.n == n) {
                L.cz = epi == EPI_STORE ? lv.cz_st : lv.cz;
                L.ts = epi == EPI_STORE ? lv.ts_st : lv.ts;
            }
    }
    return L;
}

int op(rk_ctx* c, int k, int dtype, int epi, const Coeffs& cf, const void* u, void* v,
       const void* b, const void* xo, int n, int s0, int ns, double ca, double cb,
       const void* u2 = nullptr, int xo_from_b = 0, double c0 = 0.0) {
    const OpLaunch L = op_launch(c, k, dtype, epi, cf, u, v, b, xo, n, s0, ns, ca, cb, u2, xo_from_b, c0);
    HIPCHK(c, launch_op(L));
    return RK_OK;
}

struct ChebCoef {
    double theta, delta, sigma;
};

ChebCoef cheb_coef(double up, double range) {
    const double lo = up / range;
    ChebCoef cc;
    cc.theta = 0.5 * (up + lo);
    cc.delta = 0.5 * (up - lo);
    cc.sigma = cc.theta / cc.delta;
    return cc;
}

// Multigrid on the deformed mesh.  The level blocks alpha_s M + beta_s K with
// the cell-size scaling of the affine coefficients taken out (the deformed
// operator integrates with the physical geometry).
void level_ab(const Level& L, int s0, int ns, double* al, double* be) {
    const double h3 = L.h * L.h * L.h;
    for (int s = 0; s < ns; ++s) {
        al[s] = L.blk.alpha[s0 + s] / h3;
        be[s] = L.blk.beta[s0 + s] / L.h;
    }
}

const void* at_slot(const void* base, size_t bytes) { return base ? (const char*)base + bytes : nullptr; }
void* at_slot(void* base, size_t bytes) { return base ? (char*)base + bytes : nullptr; }

// v = (blocks of level l) u for stages [s0, s0+ns), deformed mesh.
int dlevel_op(rk_ctx* c, int l, int s0, int ns, const void* u, void* v) {
    Level& L = c->lv[l];
    const size_t off = dsize(c->pc) * s0 * L.N3;
    double al[RK_MAX_Q], be[RK_MAX_Q];
    level_ab(L, s0, ns, al, be);
    HIPCHK(c, launch_deformed_apply(c->k, c->pc, L.n, ns, al, be, L.geo, at_slot(u, off), at_slot(u, off),
                                    at_slot(v, off), c->stream));
    return RK_OK;
}

// The Chebyshev iteration on the deformed levels: the same iterates as the
// fused affine version (x_1 = c0 D^-1 b from a zero start, the same
// three-term coefficients), with the operator applied into the level's temp
// and the update as a separate pass over stored diagonals.
int chebyshev_dmg(rk_ctx* c, int l, int s0, int ns, const void* b, void* first, void* second,
                  double up, double range, bool zero_start, int degree, void** res) {
    Level& L = c->lv[l];
    const double lo = up / range, theta = 0.5 * (up + lo), delta = 0.5 * (up - lo), sigma = theta / delta;
    const double c0 = 1.0 / theta;
    const size_t off = dsize(c->pc) * s0 * L.N3;
    double al[RK_MAX_Q], be[RK_MAX_Q];
    level_ab(L, s0, ns, al, be);
    const void* bb = at_slot(b, off);
    void* t = at_slot(L.t, off);
    void* cur;
    void* prev;
    if (zero_start) {
        HIPCHK(c, launch_cheb_vec(c->pc, at_slot(first, off), nullptr, nullptr, bb, nullptr, L.dMv, L.dKv, al, be,
                                  0.0, c0, L.N, ns, c->stream));
        cur = first;
        prev = nullptr;
    } else {
        int rc = dlevel_op(c, l, s0, ns, first, L.t);
        if (rc) return rc;
        HIPCHK(c, launch_cheb_vec(c->pc, at_slot(second, off), at_slot(first, off), nullptr, bb, t, L.dMv, L.dKv,
                                  al, be, 0.0, c0, L.N, ns, c->stream));
        cur = second;
        prev = first;
    }
    double rho = 1.0 / sigma;
    for (int j = 1; j < degree; ++j) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        const double ca = rho_new * rho, cb = 2.0 * rho_new / delta;
        int rc = dlevel_op(c, l, s0, ns, cur, L.t);
        if (rc) return rc;
        void* out = prev ? prev : (cur == first ? second : first);
        HIPCHK(c, launch_cheb_vec(c->pc, at_slot(out, off), at_slot(cur, off), prev ? at_slot(prev, off) : nullptr,
                                  bb, t, L.dMv, L.dKv, al, be, ca, cb, L.N, ns, c->stream));
        prev = cur;
        cur = out;
        rho = rho_new;
    }
    *res = cur;
    return RK_OK;
}

// Chebyshev iteration of `degree` steps on level l for stages [s0, s0+ns).
// first/second: stage-0 base pointers of the two iterate buffers.  If
// zero_start, x_0 = 0; otherwise x_0 is in `first`.  Returns the buffer that
// holds the result through *res.
int chebyshev(rk_ctx* c, int l, int s0, int ns, const void* b, void* first, void* second,
              bool zero_start, int degree, void** res) {
    Level& L = c->lv[l];
    if (c->dmg) return chebyshev_dmg(c, l, s0, ns, b, first, second, L.eig_max, c->opt.cheb_range, zero_start,
                                     degree, res);
    const ChebCoef cc = cheb_coef(L.eig_max, c->opt.cheb_range);
    const int k = c->k, dt = c->pc;
    const double c0 = 1.0 / cc.theta;          // x_1 = c0 D^-1 b from a zero start
    if (zero_start && degree == 1) {
        HIPCHK(c, launch_cheb_first(k, dt, to_stage_scal(L.blk), b, first, L.n, s0, ns, c0, c->stream));
        *res = first;
        return RK_OK;
    }
    void* cur;            // x_j
    void* prev;           // buffer of x_{j-1} (null: x_{j-1} = 0)
    bool prev_x1 = false; // x_{j-1} = x_1 = c0 D^-1 b, formed from b instead of stored
    double rho = 1.0 / cc.sigma;
    int j = 1;
    if (zero_start) {
        // x_2 straight from b: the kernel forms x_1 while it stages b
        const double rho_new = 1.0 / (2.0 * cc.sigma - rho);
        const double ca = rho_new * rho, cb = 2.0 * rho_new / cc.delta;
        int rc = op(c, k, dt, EPI_CHEB1, L.blk, b, second, b, nullptr, L.n, s0, ns, ca, cb, nullptr, 0, c0);
        if (rc) return rc;
        cur = second; prev = first; prev_x1 = true;
        rho = rho_new;
        j = 2;
    } else {
        int rc = op(c, k, dt, EPI_CHEB, L.blk, first, second, b, nullptr, L.n, s0, ns, 0.0, c0);
        if (rc) return rc;
        cur = second; prev = first;
    }
    for (; j < degree; ++j) {
        const double rho_new = 1.0 / (2.0 * cc.sigma - rho);
        const double ca = rho_new * rho, cb = 2.0 * rho_new / cc.delta;
        // x_{j+1} overwrites the buffer of x_{j-1}
        void* out = prev;
        int rc = op(c, k, dt, EPI_CHEB, L.blk, cur, out, b, prev_x1 ? nullptr : prev, L.n, s0, ns, ca, cb,
                    nullptr, prev_x1 ? 1 : 0, c0);
        if (rc) return rc;
        prev = cur;
        cur = out;
        prev_x1 = false;
        rho = rho_new;
    }
    *res = cur;
    return RK_OK;
}

int restrict_to(rk_ctx* c, int l, int s0, int ns, const void* fine) {
    Level& F = c->lv[l];
    Level& C = c->lv[l + 1];
    const size_t es = dsize(c->pc);
    // stage s owns tmp[s * tmp_stage ...] on every level, so that groups of
    // stages restricting on different levels at once never overlap
    void* tmp = (char*)c->tmp + es * s0 * c->tmp_stage;
    HIPCHK(c, launch_restrict(c->k, c->pc, (const char*)fine + es * s0 * F.N3, (char*)C.b + es * s0 * C.N3,
                              tmp, C.n, ns, F.N3, C.N3, c->stream));
    return RK_OK;
}

int prolong_add(rk_ctx* c, int l, int s0, int ns, const void* coarse, void* fine) {
    Level& F = c->lv[l];
    Level& C = c->lv[l + 1];
    const size_t es = dsize(c->pc);
    HIPCHK(c, launch_prolong_add(c->k, c->pc, (const char*)coarse + es * s0 * C.N3,
                                 (char*)fine + es * s0 * F.N3, C.n, ns, C.N3, F.N3, c->stream));
    return RK_OK;
}

// One V-cycle on level l for stages [s0, s0+ns): b -> result, using the two
// buffers first/second.  For l < last the result always lands in `second`;
// on the coarsest level in `first` for an odd coarse degree, else `second`.
// The V-cycle from level l (>= tail_level) down to the coarsest and back in
// one launch, one workgroup per stage block; the result lands in the buffer
// the multi-launch path would use.
int tail_vcycle(rk_ctx* c, int l, int s0, int ns, const void* b, void* first, void* second, void** res) {
    const int last = (int)c->lv.size() - 1;
    TailArgs a;
    a.nlev = last - l + 1;
    a.s0 = s0;
    a.dtype = c->pc;
    a.scratch = c->tail;
    a.sstride = (long long)c->tail_stage;
    a.n3max = c->lv[c->tail_level].N3;
    for (int i = 0; i < a.nlev; ++i) {
        const Level& L = c->lv[l + i];
        TailLevel& t = a.lv[i];
        t.b = i == 0 ? const_cast<void*>(b) : L.b;
        t.x = i == 0 ? first : L.x;
        t.y = i == 0 ? second : L.y;
        t.N3 = L.N3;
        t.n = L.n;
        t.degree = l + i == last ? c->opt.coarse_cheb_degree : c->opt.cheb_degree;
        const ChebCoef cc = cheb_coef(L.eig_max, c->opt.cheb_range);
        t.theta = cc.theta;
        t.delta = cc.delta;
        t.sigma = cc.sigma;
        for (int q = 0; q < RK_MAX_Q; ++q) { t.alpha[q] = L.blk.alpha[q]; t.beta[q] = L.blk.beta[q]; }
    }
    HIPCHK(c, launch_tail_vcycle(c->k, a, ns, c->stream));
    *res = (a.nlev > 1 || c->opt.coarse_cheb_degree % 2 == 0) ? second : first;
    return RK_OK;
}

int vcycle_level(rk_ctx* c, int l, int s0, int ns, const void* b, void* first, void* second, void** res) {
    const int last = (int)c->lv.size() - 1;
    if (c->tail_level >= 0 && l >= c->tail_level) return tail_vcycle(c, l, s0, ns, b, first, second, res);
    if (l == last) return chebyshev(c, l, s0, ns, b, first, second, true, c->opt.coarse_cheb_degree, res);
    Level& L = c->lv[l];
    void* pre = nullptr;
    int rc = chebyshev(c, l, s0, ns, b, first, second, true, c->opt.cheb_degree, &pre);
    if (rc) return rc;
    void* spare = (pre == first) ? second : first;
    // residual into the spare buffer
    if (c->dmg) {
        rc = dlevel_op(c, l, s0, ns, pre, spare);
        if (rc) return rc;
        const size_t off = dsize(c->pc) * s0 * L.N3;
        HIPCHK(c, launch_resid_vec(c->pc, at_slot(spare, off), at_slot(b, off), (long long)ns * L.N3, c->stream));
    } else {
        rc = op(c, c->k, c->pc, EPI_RESID, L.blk, pre, spare, b, nullptr, L.n, s0, ns, 0, 0);
        if (rc) return rc;
    }
    rc = restrict_to(c, l, s0, ns, spare);
    if (rc) return rc;
    Level& C = c->lv[l + 1];
    void* cres = nullptr;
    rc = vcycle_level(c, l + 1, s0, ns, C.b, C.x, C.y, &cres);
    if (rc) return rc;
    rc = prolong_add(c, l, s0, ns, cres, pre);
    if (rc) return rc;
    void* post = nullptr;
    rc = chebyshev(c, l, s0, ns, b, pre, spare, false, c->opt.cheb_degree, &post);
    if (rc) return rc;
    *res = post;
    return RK_OK;
}

// V-cycles for the blocks of slots [s0, s0+ns) on the finest level: b -> x
// (stage-0 bases of [Q][N3] buffers), with `scratch` as the second iterate
// buffer.  Batched: one launch sequence for the range; per-stage: slot by slot.
int vcycle_range(rk_ctx* c, const void* b, void* x, void* scratch, int s0, int ns) {
    const bool single = c->lv.size() == 1;
    const bool res_first = single && (c->opt.coarse_cheb_degree % 2 == 1);
    void* first = res_first ? x : scratch;
    void* second = res_first ? scratch : x;
    const int ng = c->N3 * ns >= kSplitMin ? std::min(c->opt.vc_streams, ns) : 1;
    if (ng >= 2 && c->opt.mode == RK_BATCHED) {
        if (!c->ev_fork) HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
        hipStream_t main = c->stream;
        int rc = RK_OK;
        for (int g = 0, sg = s0; g < ng && rc == RK_OK; ++g) {
            const int cnt = ns / ng + (g < ns % ng ? 1 : 0);
            if (g > 0) {
                if (!c->aux_stream[g]) {
                    HIPCHK(c, hipStreamCreateWithFlags(&c->aux_stream[g], hipStreamNonBlocking));
                    HIPCHK(c, hipEventCreateWithFlags(&c->ev_join[g], hipEventDisableTiming));
                }
                HIPCHK(c, hipStreamWaitEvent(c->aux_stream[g], c->ev_fork, 0));
                c->stream = c->aux_stream[g];
            }
            void* res = nullptr;
            rc = vcycle_level(c, 0, sg, cnt, b, first, second, &res);
            if (rc == RK_OK && res != x) rc = fail(c, RK_EHIP, "internal: V-cycle result buffer");
            if (g > 0) {
                c->stream = main;
                if (rc == RK_OK) {
                    HIPCHK(c, hipEventRecord(c->ev_join[g], c->aux_stream[g]));
                    HIPCHK(c, hipStreamWaitEvent(main, c->ev_join[g], 0));
                }
            }
            sg += cnt;
        }
        return rc;
    }
    const int groups = c->opt.mode == RK_BATCHED ? 1 : ns;
    const int per = c->opt.mode == RK_BATCHED ? ns : 1;
    for (int g = 0; g < groups; ++g) {
        void* res = nullptr;
        int rc = vcycle_level(c, 0, s0 + g * per, per, b, first, second, &res);
        if (rc) return rc;
        if (res != x) return fail(c, RK_EHIP, "internal: V-cycle result buffer");
    }
    return RK_OK;
}

// V-cycles for all Q blocks on the finest level: b -> x (both [Q][N3]).
int vcycle_all(rk_ctx* c, const void* b, void* x) {
    return vcycle_range(c, b, x, c->lv[0].y, 0, c->Q);
}

// The block solves of PRESB (eq. presb:p) on the fixed buffers, F.b -> F.x
// in slots: g1 = V(H)(F.b) on slots [0, nb) (the pairs' r_re + r_im and the
// real block), then f2 = F.b - Im(lam) M g1 on slots [nb, Q) into F.y, then
// g2 = V(H)(f2) on slots [nb, Q) (F.b serves as scratch).
int presb_blocks(rk_ctx* c) {
    Level& F = c->lv[0];
    const int nb = c->tab.nb, np = c->tab.npair;
    int rc = vcycle_range(c, F.b, F.x, F.y, 0, nb);
    if (rc || np == 0) return rc;
    const size_t es = dsize(c->pc);
    if (c->dmg) {
        // F.y[nb + j] = Im(lam_j) M g1_j on the deformed mesh, then F.b - F.y
        double al[RK_MAX_Q], be[RK_MAX_Q];
        for (int j = 0; j < np; ++j) { al[j] = c->tab.clam_im[j]; be[j] = 0.0; }
        void* fy = at_slot(F.y, es * nb * F.N3);
        HIPCHK(c, launch_deformed_apply(c->k, c->pc, F.n, np, al, be, F.geo, F.x, F.x, fy, c->stream));
        HIPCHK(c, launch_resid_vec(c->pc, fy, at_slot(F.b, es * nb * F.N3), (long long)np * F.N3, c->stream));
    } else {
        // input slot j feeds output slot nb + j: shift the input base by -nb slots
        const void* g1 = (const void*)((uintptr_t)F.x - (uintptr_t)(es * nb * F.N3));
        rc = op(c, c->k, c->pc, EPI_RESID, c->presb_m, g1, F.y, F.b, nullptr, F.n, nb, np, 0, 0);
        if (rc) return rc;
    }
    return vcycle_range(c, F.y, F.x, F.b, nb, np);
}

// The block solves of the preconditioner on F.b -> F.x.
int blocks_eager(rk_ctx* c) {
    return c->cplx ? presb_blocks(c) : vcycle_all(c, c->lv[0].b, c->lv[0].x);
}

// Block solves F.b -> F.x: replay of the captured graph, or eager launches
// (timing mode, or capture unavailable).
int run_blocks(rk_ctx* c) {
    if (c->opt.timing || c->vc_graph < 0) return blocks_eager(c);
    if (c->vc_graph == 0) {
        c->vc_graph = -1;
        if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return blocks_eager(c);
        }
        if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return blocks_eager(c);
        }
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        const int rc = blocks_eager(c);
        c->stream = user;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (rc == RK_OK && e == hipSuccess && g) e = hipGraphInstantiate(&c->vc_exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (rc != RK_OK || e != hipSuccess || !c->vc_exec) {
            (void)hipGetLastError();
            c->vc_exec = nullptr;
            return blocks_eager(c);
        }
        c->vc_graph = 1;
    }
    HIPCHK(c, hipGraphLaunch(c->vc_exec, c->stream));
    return RK_OK;
}

// z = P^-1 r on fp64 [Q][N3] vectors: eq. (irk:P) for the Crout method,
// PRESB on slot vectors (eq. presb:p) for the complex method.  If m is given,
// m = (A^-1 (x) I) z, respectively (Lam_r (x) I) z, is written in the same
// pass (the mass-term input of the Krylov operator).  r_scale: per-group
// scales of r (r_scale[group of slot j] multiplies slot j), or null.
int precondition(rk_ctx* c, const double* r, double* z, double* m = nullptr,
                 const double* r_scale = nullptr) {
    Level& F = c->lv[0];
    const int in = c->cplx ? kMixPin : kMixSinv;
    const int out = c->cplx ? kMixPout : kMixS;
    const int out2 = c->cplx ? kMixLamPout : kMixAinvS;
    {
        Timer t(c, C_BASIS);
        HIPCHK(c, launch_stage_mix(RK_FP64, r, c->pc, F.b, c->mix + in, c->Q, c->Q, c->N, c->stream,
                                   nullptr, nullptr, r_scale, &c->slot_group));
    }
    {
        Timer t(c, C_BLOCKS);
        int rc = run_blocks(c);
        if (rc) return rc;
    }
    Timer t(c, C_BASIS);
    HIPCHK(c, launch_stage_mix(c->pc, F.x, RK_FP64, z, c->mix + out, c->Q, c->Q, c->N, c->stream, m,
                               m ? c->mix + out2 : nullptr));
    return RK_OK;
}

// Largest eigenvalue of D^-1 A per level (max over blocks), by power
// iteration with a Rayleigh-quotient estimate.
int estimate_eigs(rk_ctx* c) {
    const int Q = c->Q, dt = c->pc;
    for (size_t l = 0; l < c->lv.size(); ++l) {
        Level& L = c->lv[l];
        if (L.N <= 2) { L.eig_max = 1.0; continue; }
        HIPCHK(c, launch_random_fill(dt, L.x, L.N, Q, 12345u + 977u * (unsigned)l, c->stream));
        StageScal sc = to_stage_scal(L.blk);
        if (c->dmg) level_ab(L, 0, Q, sc.alpha, sc.beta);
        for (int it = 0; it < c->opt.eig_iterations; ++it) {
            int rc = c->dmg ? dlevel_op(c, (int)l, 0, Q, L.x, L.y)
                            : op(c, c->k, dt, EPI_STORE, L.blk, L.x, L.y, nullptr, nullptr, L.n, 0, Q, 0, 0);
            if (rc) return rc;
            HIPCHK(c, launch_power_partial(c->k, dt, sc, L.x, L.y, L.b, L.n, Q, c->part, kRedBlocks, c->stream,
                                           c->dmg ? L.dMv : nullptr, c->dmg ? L.dKv : nullptr));
            HIPCHK(c, launch_reduce(c->part, kRedBlocks, 3 * Q, c->scal, 0, c->stream));
            if (it + 1 < c->opt.eig_iterations)
                HIPCHK(c, launch_power_normalize(dt, L.b, L.x, c->scal, L.N, Q, c->stream));
        }
        double red[3 * RK_MAX_Q];
        HIPCHK(c, hipMemcpyAsync(red, c->scal, sizeof(double) * 3 * Q, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double mx = 0.0;
        for (int s = 0; s < Q; ++s)
            if (red[3 * s + 1] > 0) mx = std::max(mx, red[3 * s] / red[3 * s + 1]);
        L.eig_max = mx > 0 ? c->opt.eig_safety * mx : 1.0;
    }
    return RK_OK;
}

// Average time of `reps` launches of fn() on the context stream (HIP events).
template <typename F>
int time_launches(rk_ctx* c, int reps, F&& fn, float* ms) {
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    int rc = fn();                                   // warm-up
    if (rc == RK_OK) rc = hipEventRecord(a, c->stream) == hipSuccess ? RK_OK : RK_EHIP;
    for (int i = 0; i < reps && rc == RK_OK; ++i) rc = fn();
    if (rc == RK_OK) rc = hipEventRecord(b, c->stream) == hipSuccess ? RK_OK : RK_EHIP;
    if (rc == RK_OK) rc = hipEventSynchronize(b) == hipSuccess ? RK_OK : RK_EHIP;
    if (rc == RK_OK) rc = hipEventElapsedTime(ms, a, b) == hipSuccess ? RK_OK : RK_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != RK_OK) return fail(c, RK_EHIP, "autotune timing failed");
    *ms /= reps;
    return RK_OK;
}

// The tile autotuner: per level, the z-chunk length of the diagonal-mix
// operator in the preconditioner precision (on the level's buffers, with the
// V-cycle's stage count), and for the fine-level fp64 pair operator of the
// Krylov method.  Candidates 1, 2, 4, 8, 16 elements are timed in three
// interleaved rounds of four launches each, after untimed launches that bring
// the clocks up; the candidate with the lowest mean over its rounds wins (a
// single lucky round does not).  The operator's results do not depend on the
// choice (the work decomposition changes, the arithmetic of every output
// does not).
// Times the launches with every z-chunk of 1..16 elements and, if ts_slot is
// given, both tile shapes: three interleaved rounds of four launches each
// after a warm-up; the lowest mean wins.
int pick_chunk(rk_ctx* c, int* cz_slot, const std::function<int()>& launch, int* ts_slot = nullptr) {
    static const int cand[] = {1, 2, 4, 8, 16};
    constexpr int ncz = 5, rounds = 3;
    const int nts = ts_slot ? 2 : 1;
    float sum[2 * ncz] = {};
    *cz_slot = 0;                                    // warm-up with the size heuristic
    if (ts_slot) *ts_slot = 0;
    for (int i = 0; i < 8; ++i)
        if (int rc = launch()) return rc;
    for (int r = 0; r < rounds; ++r)
        for (int t = 0; t < nts; ++t)
            for (int i = 0; i < ncz; ++i) {
                *cz_slot = cand[i];
                if (ts_slot) *ts_slot = t;
                float ms = 0.f;
                if (int rc = time_launches(c, 4, launch, &ms)) return rc;
                sum[t * ncz + i] += ms;
            }
    int pick = 0;
    for (int i = 1; i < nts * ncz; ++i)
        if (sum[i] < sum[pick]) pick = i;
    *cz_slot = cand[pick % ncz];
    if (ts_slot) *ts_slot = pick / ncz;
    return RK_OK;
}

int autotune(rk_ctx* c) {
    const int ns = c->opt.mode == RK_BATCHED ? c->Q : 1;
    // the second tile shape exists for the fp32 diagonal-mix kernels only
    const bool shapes = c->pc == RK_FP32;
    for (size_t l = 0; l < c->lv.size() && !c->dmg; ++l) {
        Level& L = c->lv[l];
        HIPCHK(c, launch_random_fill(c->pc, L.x, L.N, c->Q, 777u + (unsigned)l, c->stream));
        HIPCHK(c, launch_random_fill(c->pc, L.b, L.N, c->Q, 999u + (unsigned)l, c->stream));
        // the V-cycle epilogues, timed as the Chebyshev update (the most frequent)
        int rc = pick_chunk(c, &L.cz, [&] {
            return op(c, c->k, c->pc, EPI_CHEB, L.blk, L.x, L.y, L.b, nullptr, L.n, 0, ns, 0.5, 0.5);
        }, shapes ? &L.ts : nullptr);
        if (rc) return rc;
        rc = pick_chunk(c, &L.cz_st, [&] {
            return op(c, c->k, c->pc, EPI_STORE, L.blk, L.x, L.y, nullptr, nullptr, L.n, 0, ns, 0, 0);
        }, shapes ? &L.ts_st : nullptr);
        if (rc) return rc;
    }
    // fine-level fp64 pair operator (mass input in mbuf, stiffness input in w)
    HIPCHK(c, launch_random_fill(RK_FP64, c->mbuf, c->N, c->Q, 4242u, c->stream));
    HIPCHK(c, launch_random_fill(RK_FP64, c->w, c->N, c->Q, 4243u, c->stream));
    if (!c->deformed) {
        int rc = pick_chunk(c, &c->cz_pair, [&] {
            return op(c, c->k, RK_FP64, EPI_STORE, c->form[F_CALA], c->mbuf, c->kv, nullptr, nullptr, c->n, 0, c->Q,
                      0, 0, c->w);
        });
        if (rc) return rc;
    }
    return RK_OK;
}

// Arnoldi step j for every group (independent system) at once.  The basis is
// stored unnormalised, V_i = sig[i][g] Vhat_i on group g, with the scale
// factors sig on the device, so no separate normalisation pass is needed.
// w = A z_j is orthogonalised against V_0..V_j by classical Gram-Schmidt
// (one fused dot pass and one update pass); a second pass runs when in some
// group the projection cancelled all but 1e-4 of ||w||^2.  The result goes to
// Vhat_{j+1} and sig[j+1][g] = 1/||Vhat_{j+1}|| on g.  Returns, per group g,
// hcol[g * (restart + 2) + i] = h_ij (i <= j) and h_{j+1,j} = ||w_orth||.
int arnoldi_orth(rk_ctx* c, int j, double* hcol) {
    const int nv = j + 1, ng = c->ng, NS = c->nscal, hs = c->opt.restart + 2;
    double* Vn = c->V + (long long)nv * c->ld;
    double* host = c->host_scal.data();
    double* sig_n = c->sig + (long long)nv * kSigStride;
    HIPCHK(c, launch_dots(c->V, nv, c->ld, c->w, c->seg, 1, c->part, kRedBlocks, c->stream));
    HIPCHK(c, launch_reduce(c->part, kRedBlocks, nv + 1, c->scal, 0, c->stream, c->sig, nv, nullptr, ng, NS));
    HIPCHK(c, launch_gs_update(c->V, nv, c->ld, c->scal, NS, c->sig, c->w, Vn, c->seg, c->part, kRedBlocks,
                               c->stream));
    HIPCHK(c, launch_reduce(c->part, kRedBlocks, 1, c->scal + nv + 1, 0, c->stream, nullptr, 0, sig_n, ng, NS));
    HIPCHK(c, hipMemcpyAsync(host, c->scal, sizeof(double) * NS * ng, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bool again = false;
    for (int g = 0; g < ng; ++g) {
        const double* hg = host + (long long)g * NS;
        for (int i = 0; i < nv; ++i) hcol[g * hs + i] = hg[i];
        hcol[g * hs + nv] = hg[nv + 1];          // ||w_orth||^2 for now
        if (hg[nv + 1] < 1e-4 * hg[nv]) again = true;
    }
    if (again) {
        HIPCHK(c, launch_dots(c->V, nv, c->ld, Vn, c->seg, 0, c->part, kRedBlocks, c->stream));
        HIPCHK(c, launch_reduce(c->part, kRedBlocks, nv, c->scal2, 0, c->stream, c->sig, nv, nullptr, ng, NS));
        HIPCHK(c, launch_gs_update(c->V, nv, c->ld, c->scal2, NS, c->sig, Vn, Vn, c->seg, c->part, kRedBlocks,
                                   c->stream));
        HIPCHK(c, launch_reduce(c->part, kRedBlocks, 1, c->scal2 + nv, 0, c->stream, nullptr, 0, sig_n, ng, NS));
        HIPCHK(c, hipMemcpyAsync(host, c->scal2, sizeof(double) * NS * ng, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int g = 0; g < ng; ++g) {
            const double* hg = host + (long long)g * NS;
            for (int i = 0; i < nv; ++i) hcol[g * hs + i] += hg[i];
            hcol[g * hs + nv] = hg[nv];
        }
    }
    for (int g = 0; g < ng; ++g) hcol[g * hs + nv] = std::sqrt(std::max(hcol[g * hs + nv], 0.0));
    return RK_OK;
}

// ||x||^2 per group on the host (out[g]); with inv_sqrt, also 1/||x|| per
// group into those device scalars (inv_sqrt[g]).
int group_norm2(rk_ctx* c, const double* x, double* out, double* inv_sqrt = nullptr) {
    HIPCHK(c, launch_dots(nullptr, 0, 0, x, c->seg, 1, c->part, kRedBlocks, c->stream));
    HIPCHK(c, launch_reduce(c->part, kRedBlocks, 1, c->scal, 0, c->stream, nullptr, 0, inv_sqrt, c->ng, c->nscal));
    double* host = c->host_scal.data();
    HIPCHK(c, hipMemcpyAsync(host, c->scal, sizeof(double) * c->nscal * c->ng, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int g = 0; g < c->ng; ++g) out[g] = host[(long long)g * c->nscal];
    return RK_OK;
}

// v_s = alpha_s M um_s + beta_s K u_s on the deformed mesh (fp64, ns stages).
int deformed_op(rk_ctx* c, int ns, const double* alpha, const double* beta, const void* um, const void* u,
                void* v) {
    HIPCHK(c, launch_deformed_apply(c->k, RK_FP64, c->n, ns, alpha, beta, c->geo, um, u, v, c->stream));
    return RK_OK;
}

// v = (D (x) M + tau I (x) K) u given m = (D (x) I) u, where D = A^-1 (eq.
// irk:A, Crout method) or Lam_r (complex method); with b, v = b - (...) u.
int apply_krylov(rk_ctx* c, const double* u, const double* m, double* v, const double* b) {
    Timer t(c, C_VMULT);
    if (c->deformed) {
        double al[RK_MAX_Q], be[RK_MAX_Q];
        for (int s = 0; s < c->Q; ++s) { al[s] = 1.0; be[s] = c->tau; }
        int rc = deformed_op(c, c->Q, al, be, m, u, v);
        if (rc || !b) return rc;
        HIPCHK(c, launch_sub_from(v, b, (long long)c->Q * c->N3, c->stream));
        return RK_OK;
    }
    return op(c, c->k, RK_FP64, b ? EPI_RESID : EPI_STORE, c->form[c->cplx ? F_CBLK : F_CALA], m, v, b, nullptr,
              c->n, 0, c->Q, 0, 0, u);
}

// Right-preconditioned flexible GMRES (Saad, Alg. 9.6; zero initial guess,
// restarts of length m, Givens rotations) on c->ng independent systems in
// lock step: the Krylov operator is block diagonal over the groups, every
// group has its own basis scales, Hessenberg matrix, rotations and
// convergence test ||r_g|| <= rtol ||rhs_g||, and all groups share every
// kernel launch.  A group that has converged within a cycle keeps running
// (its extra columns are not used); at a restart its start vector is scaled
// to zero, so it contributes nothing further.  rhs: c->rhs; solution: c->kv.
int gmres(rk_ctx* c, rk_stats& st, bool& converged) {
    const int ng = c->ng, m = c->opt.restart, hs = m + 2;
    const long long qn = (long long)c->Q * c->N3;
    std::vector<double> bn(ng), rn(ng), sig0(ng);
    int rc = group_norm2(c, c->rhs, bn.data());
    if (rc) return rc;
    for (auto& v : bn) v = std::sqrt(v);
    HIPCHK(c, launch_fill(RK_FP64, c->kv, qn, 0.0, c->stream));
    // the residual of each restart cycle lives in Vhat_0 (k_0 = 0: r = rhs)
    HIPCHK(c, launch_copy(RK_FP64, c->rhs, c->V, qn, c->stream));
    const int vc_per_it = c->opt.mode == RK_BATCHED ? (c->cplx && c->tab.npair > 0 ? 2 : 1) : c->Q;
    std::vector<char> active(ng), done(ng);
    std::vector<int> jd(ng);
    std::vector<double> H((size_t)ng * (m + 1) * m), cs((size_t)ng * m), sn((size_t)ng * m), gv((size_t)ng * (m + 1)),
        hcol((size_t)ng * hs), yv((size_t)ng * c->nscal, 0.0);
    int its = 0, vcyc = 0;
    bool fresh = false;   // rn holds the norms of the current residual
    for (int g = 0; g < ng; ++g) active[g] = bn[g] > 0.0;
    while (its < c->opt.max_iter) {
        rc = group_norm2(c, c->V, rn.data());
        if (rc) return rc;
        fresh = true;
        bool any = false;
        for (int g = 0; g < ng; ++g) {
            rn[g] = std::sqrt(rn[g]);
            if (active[g] && rn[g] <= c->opt.rtol * bn[g]) active[g] = 0;
            sig0[g] = active[g] ? 1.0 / rn[g] : 0.0;
            any = any || active[g];
        }
        if (!any) break;
        HIPCHK(c, hipMemcpyAsync(c->sig, sig0.data(), sizeof(double) * ng, hipMemcpyHostToDevice, c->stream));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(gv.begin(), gv.end(), 0.0);
        for (int g = 0; g < ng; ++g) {
            gv[(size_t)g * (m + 1)] = active[g] ? rn[g] : 0.0;
            done[g] = !active[g];
            jd[g] = 0;
        }
        int jmax = 0;
        for (int j = 0; j < m && its < c->opt.max_iter; ++j) {
            rc = precondition(c, c->V + (long long)j * c->ld, c->Z + (long long)j * c->ld, (double*)c->mbuf,
                              c->sig + (long long)j * kSigStride);
            if (rc) return rc;
            vcyc += vc_per_it;
            rc = apply_krylov(c, c->Z + (long long)j * c->ld, (const double*)c->mbuf, c->w, nullptr);
            if (rc) return rc;
            {
                Timer t(c, C_REST);
                rc = arnoldi_orth(c, j, hcol.data());
                if (rc) return rc;
            }
            ++its;
            jmax = j + 1;
            bool all = true;
            for (int g = 0; g < ng; ++g) {
                if (done[g]) continue;
                double* Hg = H.data() + (size_t)g * (m + 1) * m;
                double *csg = cs.data() + (size_t)g * m, *sng = sn.data() + (size_t)g * m;
                double* gg = gv.data() + (size_t)g * (m + 1);
                const double* hc = hcol.data() + (size_t)g * hs;
                for (int i = 0; i <= j + 1; ++i) Hg[(size_t)i * m + j] = hc[i];
                for (int i = 0; i < j; ++i) {
                    const double a = Hg[(size_t)i * m + j], b = Hg[(size_t)(i + 1) * m + j];
                    Hg[(size_t)i * m + j] = csg[i] * a + sng[i] * b;
                    Hg[(size_t)(i + 1) * m + j] = -sng[i] * a + csg[i] * b;
                }
                const double a = Hg[(size_t)j * m + j], b = Hg[(size_t)(j + 1) * m + j];
                const double d = std::hypot(a, b);
                csg[j] = d > 0 ? a / d : 1.0;
                sng[j] = d > 0 ? b / d : 0.0;
                Hg[(size_t)j * m + j] = d;
                Hg[(size_t)(j + 1) * m + j] = 0.0;
                gg[j + 1] = -sng[j] * gg[j];
                gg[j] = csg[j] * gg[j];
                jd[g] = j + 1;
                if (c->cplx) ++st.block_iterations[g];
                if (std::fabs(gg[j + 1]) <= c->opt.rtol * bn[g] || hc[j + 1] == 0.0) done[g] = 1;
                else all = false;
            }
            if (all) break;
        }
        // y_g = H_g^-1 g_g (upper triangular) on the group's jd columns, k += Z y
        std::fill(yv.begin(), yv.end(), 0.0);
        for (int g = 0; g < ng; ++g) {
            const double* Hg = H.data() + (size_t)g * (m + 1) * m;
            const double* gg = gv.data() + (size_t)g * (m + 1);
            double* yg = yv.data() + (size_t)g * c->nscal;
            for (int i = jd[g] - 1; i >= 0; --i) {
                double s = gg[i];
                for (int l = i + 1; l < jd[g]; ++l) s -= Hg[(size_t)i * m + l] * yg[l];
                yg[i] = s / Hg[(size_t)i * m + i];
            }
        }
        {
            Timer t(c, C_REST);
            HIPCHK(c, hipMemcpyAsync(c->ycoef, yv.data(), sizeof(double) * yv.size(), hipMemcpyHostToDevice,
                                     c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            HIPCHK(c, launch_combine(c->kv, RK_FP64, c->Z, jmax, c->ld, c->ycoef, c->nscal, c->seg, c->stream));
        }
        // true residual r = rhs - A k
        HIPCHK(c, launch_stage_mix(RK_FP64, c->kv, RK_FP64, c->mbuf, c->mix + (c->cplx ? kMixCLam : kMixAinv),
                                   c->Q, c->Q, c->N, c->stream));
        rc = apply_krylov(c, c->kv, (const double*)c->mbuf, c->V, c->rhs);
        if (rc) return rc;
        fresh = false;
    }
    if (!fresh) {
        rc = group_norm2(c, c->V, rn.data());
        if (rc) return rc;
        for (auto& v : rn) v = std::sqrt(v);
    }
    converged = true;
    double worst = 0.0;
    for (int g = 0; g < ng; ++g) {
        const double rel = bn[g] > 0 ? rn[g] / bn[g] : 0.0;
        worst = std::max(worst, rel);
        if (bn[g] > 0 && rn[g] > c->opt.rtol * bn[g]) converged = false;
    }
    st.iterations = its;
    st.vcycles = vcyc;
    st.rel_residual = worst;
    return RK_OK;
}

}  // namespace

namespace rk {
int report_free_error(int code, const std::string& msg) { return fail(nullptr, code, msg); }
}  // namespace rk

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void rk_default_options(rk_options* o) {
    if (!o) return;
    o->precision = RK_PREC_FP64;
    o->mode = RK_BATCHED;
    o->rtol = 1e-10;
    o->max_iter = 200;
    o->restart = 30;
    o->cheb_degree = 3;
    o->coarse_cheb_degree = 3;
    o->cheb_range = 15.0;
    o->eig_safety = 1.2;
    o->eig_iterations = 30;
    o->eig_max = nullptr;
    o->timing = 0;
    o->method = RK_METHOD_CROUT;
    o->deform = 0.0;
    o->autotune = 1;
    o->deform_mg = 1;
    o->vc_streams = 2;
    o->z_chunk = 0;
    o->tile_shape = 0;
    o->tail_nodes = 17 * 17 * 17;
}

int rk_workspace_bytes(const rk_mesh* mesh, int degree, int Q, const rk_options* opt, size_t* bytes) {
    if (!bytes) return fail(nullptr, RK_EINVAL, "bytes is NULL");
    rk_ctx c;
    int rc = setup_sizes(c, mesh, degree, Q, opt);
    if (rc) return rc;
    *bytes = carve(c, nullptr);
    return RK_OK;
}

int rk_create(const rk_mesh* mesh, int degree, int Q, double tau, const rk_options* opt, void* d_workspace,
              size_t workspace_bytes, void* hip_stream, rk_ctx** out) {
    if (!out) return fail(nullptr, RK_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(tau > 0.0)) return fail(nullptr, RK_EINVAL, "tau must be positive");
    rk_ctx* c = new rk_ctx();
    int rc = setup_sizes(*c, mesh, degree, Q, opt);
    if (rc) { delete c; return rc; }
    c->tau = tau;
    if (c->opt.eig_max) {
        c->eig_user.assign(c->opt.eig_max, c->opt.eig_max + c->lv.size());
        for (double v : c->eig_user)
            if (!(v > 0.0)) { delete c; return fail(nullptr, RK_EINVAL, "eig_max entries must be positive"); }
    }
    c->opt.eig_max = nullptr;
    const size_t need = carve(*c, nullptr);
    if (!d_workspace || workspace_bytes < need) {
        delete c;
        return fail(nullptr, RK_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    if (((uintptr_t)d_workspace) % kAlign) { delete c; return fail(nullptr, RK_EINVAL, "workspace not 256-byte aligned"); }
    carve(*c, (char*)d_workspace);
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fail(nullptr, RK_EHIP, "no HIP device"); }
    c->host_scal.assign((size_t)c->nscal * ((Q + 1) / 2), 0.0);
    std::string msg;
    if (!build_tableau(Q, c->tab, msg)) { delete c; return fail(nullptr, RK_EINVAL, msg); }
    build_element(degree, c->el);
    for (int f = 0; f < F_NFORMS; ++f) c->form[f] = make_coeffs(*c, c->h, f);
    for (auto& L : c->lv) L.blk = make_coeffs(*c, L.h, F_BLOCKS);
    {
        const Tableau& t = c->tab;
        const double h3 = c->h * c->h * c->h;
        for (int j = 0; j < t.npair; ++j) c->presb_m.alpha[t.nb + j] = t.clam_im[j] * h3;
        // Krylov systems: one over all stages, or one per block of slots
        c->ng = c->cplx ? t.nb : 1;
        Segs sg;
        sg.ngroup = c->ng;
        int q = 0;
        for (int g = 0; g < c->ng; ++g) {
            sg.first[g] = q;
            if (!c->cplx) { sg.off[q] = 0; sg.len[q] = (long long)Q * c->N3; ++q; continue; }
            const int slots[2] = {g, t.nb + g};
            for (int i = 0; i < (g < t.npair ? 2 : 1); ++i) {
                sg.off[q] = (long long)slots[i] * c->N3;
                sg.len[q] = c->N3;
                c->slot_group.v[slots[i]] = g;
                ++q;
            }
        }
        sg.first[c->ng] = q;
        c->seg = sg;
    }
    // small Q x Q mixing data: S^-1, S, the right-hand-side coefficients, and
    // the slot mixes of the complex method
    std::vector<double> mix(kMixSlots * 81, 0.0);
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            double as = 0.0;
            for (int l = 0; l < Q; ++l) as += c->tab.Ainv[i * Q + l] * c->tab.S[l * Q + j];
            mix[kMixAinvS + i * Q + j] = as;
        }
    for (int i = 0; i < Q * Q; ++i) {
        mix[kMixSinv + i] = c->tab.Sinv[i];
        mix[kMixS + i] = c->tab.S[i];
        mix[kMixAinv + i] = c->tab.Ainv[i];
        mix[kMixA + i] = c->tab.A[i];
        mix[kMixCLam + i] = c->tab.CLam[i];
    }
    {
        // PRESB (eq. presb:p) around the two block solves: per pair j the
        // inputs are (r_re + r_im, r_im) on slots (j, nb + j) and the outputs
        // (g1 - g2, g2); the real block passes through.  LamPout = Lam_r Pout.
        const Tableau& t = c->tab;
        double* pin = mix.data() + kMixPin;
        double* pout = mix.data() + kMixPout;
        for (int s = 0; s < Q; ++s) { pin[s * Q + s] = 1.0; pout[s * Q + s] = 1.0; }
        for (int j = 0; j < t.npair; ++j) {
            pin[j * Q + t.nb + j] = 1.0;
            pout[j * Q + t.nb + j] = -1.0;
        }
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j) {
                double acc = 0.0;
                for (int l = 0; l < Q; ++l) acc += t.CLam[i * Q + l] * pout[l * Q + j];
                mix[kMixLamPout + i * Q + j] = acc;
            }
    }
    hipError_t e = hipMemcpyAsync(c->mix, mix.data(), mix.size() * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->deformed)
        e = launch_deformed_geometry(c->k, RK_FP64, c->n, c->opt.deform, c->geo, c->stream);
    for (size_t l = 0; c->dmg && l < c->lv.size() && e == hipSuccess; ++l) {
        Level& L = c->lv[l];
        e = launch_deformed_geometry(c->k, c->pc, L.n, c->opt.deform, L.geo, c->stream);
        if (e == hipSuccess) e = launch_deformed_diag(c->k, c->pc, L.n, L.geo, L.dMv, L.dKv, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { delete c; return fail(nullptr, RK_EHIP, hipGetErrorString(e)); }
    if (!c->eig_user.empty()) {
        for (size_t l = 0; l < c->lv.size(); ++l) c->lv[l].eig_max = c->eig_user[l];
    } else if ((rc = estimate_eigs(c))) {
        g_create_error = c->err; delete c; return rc;
    }
    if (c->opt.z_chunk > 0) {   // a fixed chunk for every launch (reported by rk_info)
        for (auto& lv : c->lv) {
            lv.cz = lv.cz_st = c->opt.z_chunk;
            lv.ts = lv.ts_st = c->pc == RK_FP32 ? c->opt.tile_shape : 0;
        }
        c->cz_pair = c->opt.z_chunk;
    } else if (c->opt.autotune && (rc = autotune(c))) {
        g_create_error = c->err; delete c; return rc;
    }
    // the private streams and events of split V-cycles, made here rather
    // than on first use (which may fall inside a graph capture)
    const int groups = c->opt.mode == RK_BATCHED && c->N3 * c->Q >= kSplitMin ? std::min(c->opt.vc_streams, c->Q)
                                                                          : 1;
    if (groups >= 2) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    for (int g = 1; g < groups && e == hipSuccess; ++g) {
        e = hipStreamCreateWithFlags(&c->aux_stream[g], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join[g], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        rk_destroy(c);
        return fail(nullptr, RK_EHIP, hipGetErrorString(e));
    }
    *out = c;
    return RK_OK;
}

int rk_destroy(rk_ctx* c) {
    if (!c) return RK_EINVAL;
    // queued work of the context may still use the workspace the caller
    // frees after this call
    (void)hipStreamSynchronize(c->stream);
    for (auto& e : c->event_pool) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    if (c->vc_exec) (void)hipGraphExecDestroy(c->vc_exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (int g = 0; g < RK_MAX_Q; ++g) {
        if (c->aux_stream[g]) (void)hipStreamDestroy(c->aux_stream[g]);
        if (c->ev_join[g]) (void)hipEventDestroy(c->ev_join[g]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    delete c;
    return RK_OK;
}

int rk_info(const rk_ctx* c, rk_info_t* o) {
    if (!c || !o) return RK_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->N = c->N; o->n_cells = c->n; o->degree = c->k; o->Q = c->Q; o->n_levels = (int)c->lv.size();
    for (size_t l = 0; l < c->lv.size(); ++l) { o->level_cells[l] = c->lv[l].n; o->eig_max[l] = c->lv[l].eig_max; }
    o->tau = c->tau; o->h = c->h;
    const int Q = c->Q;
    for (int i = 0; i < Q * Q; ++i) {
        o->A[i] = c->tab.A[i]; o->Ainv[i] = c->tab.Ainv[i]; o->L[i] = c->tab.L[i];
        o->S[i] = c->tab.S[i]; o->Sinv[i] = c->tab.Sinv[i];
    }
    for (int i = 0; i < Q; ++i) { o->b[i] = c->tab.b[i]; o->c[i] = c->tab.c[i]; o->lambda[i] = c->tab.lam[i]; }
    for (int i = 0; i <= c->k; ++i) o->nodes[i] = c->el.nodes[i];
    o->n_blocks = c->tab.nb;
    o->n_pairs = c->tab.npair;
    for (int i = 0; i < Q; ++i) { o->clam_re[i] = c->tab.clam_re[i]; o->clam_im[i] = c->tab.clam_im[i]; }
    for (int i = 0; i < Q * Q; ++i) { o->T[i] = c->tab.CT[i]; o->U[i] = c->tab.CU[i]; }
    for (size_t l = 0; l < c->lv.size(); ++l) {
        o->level_cz[l] = c->lv[l].cz;
        o->level_ts[l] = c->lv[l].ts;
        o->level_cz_store[l] = c->lv[l].cz_st;
        o->level_ts_store[l] = c->lv[l].ts_st;
    }
    o->krylov_cz = c->cz_pair;
    o->tail_level = c->tail_level;
    return RK_OK;
}

int rk_apply_operator(rk_ctx* c, int form, int dtype, const void* u, void* v) {
    if (!c) return RK_EINVAL;
    if (!u || !v) return fail(c, RK_EINVAL, "NULL vector");
    if (form < 0 || form >= F_NFORMS) return fail(c, RK_EINVAL, "bad operator form");
    if (dtype != RK_FP64 && dtype != RK_FP32) return fail(c, RK_EINVAL, "bad dtype");
    const int ns = (form == F_K || form == F_M) ? 1 : c->Q;
    const size_t bytes = dsize(dtype) * (size_t)ns * c->N3;
    if ((const char*)u < (const char*)v + bytes && (const char*)v < (const char*)u + bytes)
        return fail(c, RK_EINVAL, "u and v overlap");
    const Coeffs& cf = c->form[form];
    if (c->deformed) {
        if (dtype != RK_FP64) return fail(c, RK_EINVAL, "a deformed-mesh context applies fp64 operators only");
        double al[RK_MAX_Q], be[RK_MAX_Q];
        if (form == F_K || form == F_M) {
            al[0] = form == F_M ? 1.0 : 0.0;
            be[0] = form == F_K ? 1.0 : 0.0;
            return deformed_op(c, 1, al, be, u, u, v);
        }
        if (form != F_CALA && form != F_CBLK)
            return fail(c, RK_EINVAL, "operator form not available on a deformed mesh");
        HIPCHK(c, launch_stage_mix(RK_FP64, u, RK_FP64, c->mbuf, c->mix + (form == F_CALA ? kMixAinv : kMixCLam),
                                   c->Q, c->Q, c->N, c->stream));
        for (int s = 0; s < c->Q; ++s) { al[s] = 1.0; be[s] = c->tau; }
        return deformed_op(c, c->Q, al, be, c->mbuf, u, v);
    }
    if (!cf.pair) return op(c, c->k, dtype, EPI_STORE, cf, u, v, nullptr, nullptr, c->n, 0, ns, 0, 0);
    // dense forms: mix the input once, then the pair operator
    const double* D = c->mix + (cf.premix == 1 ? kMixAinv : cf.premix == 2 ? kMixA : kMixCLam);
    HIPCHK(c, launch_stage_mix(dtype, u, dtype, c->mbuf, D, c->Q, c->Q, c->N, c->stream));
    const void* um = cf.premix != 2 ? c->mbuf : u;
    const void* uk = cf.premix != 2 ? u : c->mbuf;
    return op(c, c->k, dtype, EPI_STORE, cf, um, v, nullptr, nullptr, c->n, 0, ns, 0, 0, uk);
}

int rk_apply_operator_batch(rk_ctx* const* ctx, int count, int form, int dtype, const void* const* u,
                            void* const* v, void* hip_stream) {
    if (count < 1 || !ctx || !u || !v) return fail(nullptr, RK_EINVAL, "bad batch arguments");
    if (form != F_BLOCKS && form != F_K && form != F_M)
        return fail(nullptr, RK_EINVAL, "batched forms: RK_OP_BLOCKS, RK_OP_K, RK_OP_M");
    if (dtype != RK_FP64 && dtype != RK_FP32) return fail(nullptr, RK_EINVAL, "bad dtype");
    std::vector<std::pair<const char*, const char*>> in(count), out(count);
    for (int i = 0; i < count; ++i) {
        if (!ctx[i] || !u[i] || !v[i]) return fail(nullptr, RK_EINVAL, "NULL context or vector in the batch");
        if (ctx[i]->deformed) return fail(nullptr, RK_EINVAL, "the batched operator runs on affine meshes only");
        const int ns = form == F_BLOCKS ? ctx[i]->Q : 1;
        const size_t bytes = dsize(dtype) * (size_t)ns * ctx[i]->N3;
        in[i] = {(const char*)u[i], (const char*)u[i] + bytes};
        out[i] = {(const char*)v[i], (const char*)v[i] + bytes};
    }
    // no output may overlap any input or another output of the batch
    auto meet = [](const std::pair<const char*, const char*>& a, const std::pair<const char*, const char*>& b) {
        return a.first < b.second && b.first < a.second;
    };
    for (int i = 0; i < count; ++i)
        for (int j = 0; j < count; ++j)
            if (meet(out[i], in[j]) || (j < i && meet(out[i], out[j])))
                return fail(nullptr, RK_EINVAL, "an output vector of the batch overlaps another vector");
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // Problems that fill the GPU on their own take their context's tuned
    // launch; the others go into one work list per degree, in chunks of at
    // most kOpListMax problems.
    for (int k = 1; k <= RK_MAX_DEGREE; ++k) {
        std::vector<OpLaunch> list;
        for (int i = 0; i < count; ++i) {
            const rk_ctx* c = ctx[i];
            if (c->k != k) continue;
            const int ns = form == F_BLOCKS ? c->Q : 1;
            OpLaunch L = op_launch(c, k, dtype, EPI_STORE, c->form[form], u[i], v[i], nullptr, nullptr, c->n, 0, ns,
                                   0.0, 0.0);
            if ((double)ns * c->N3 >= kOpListAlone) {
                L.stream = st;
                const hipError_t e = launch_op(L);
                if (e != hipSuccess) return fail(nullptr, RK_EHIP, std::string("HIP: ") + hipGetErrorString(e));
            } else {
                list.push_back(L);
            }
        }
        for (size_t i0 = 0; i0 < list.size(); i0 += kOpListMax) {
            const int m = (int)std::min<size_t>(kOpListMax, list.size() - i0);
            const hipError_t e = launch_op_list(list.data() + i0, m, st);
            if (e != hipSuccess) return fail(nullptr, RK_EHIP, std::string("HIP: ") + hipGetErrorString(e));
        }
    }
    return RK_OK;
}

int rk_vcycle(rk_ctx* c, int dtype, const void* b, void* x) {
    if (!c) return RK_EINVAL;
    if (!b || !x) return fail(c, RK_EINVAL, "NULL vector");
    if (dtype != c->pc) return fail(c, RK_EINVAL, "dtype must match the preconditioner precision");
    const size_t bytes = dsize(dtype) * (size_t)c->Q * c->N3;
    if ((const char*)b < (const char*)x + bytes && (const char*)x < (const char*)b + bytes)
        return fail(c, RK_EINVAL, "b and x overlap");
    return vcycle_all(c, b, x);
}

int rk_apply_preconditioner(rk_ctx* c, const double* r, double* z) {
    if (!c) return RK_EINVAL;
    if (!r || !z) return fail(c, RK_EINVAL, "NULL vector");
    return precondition(c, r, z);
}

int rk_step(rk_ctx* c, double t_n, double* y, const double* G, const double* gamma, rk_stats* stats) {
    (void)t_n;
    if (!c) return RK_EINVAL;
    if (!y) return fail(c, RK_EINVAL, "y is NULL");
    if (G && !gamma) return fail(c, RK_EINVAL, "gamma is NULL while G is given");
    const int Q = c->Q;
    c->pool_used = 0;
    rk_stats st{};
    int rc;
    // Right-hand side of eq. (irk:A): rhs_i = sum_j Ainv_ij (gamma_j G - K y);
    // for the complex method directly in slots, (T (x) I) rhs.
    {
        Timer t(c, C_RHS);
        if (c->deformed) {
            const double al = 0.0, be = 1.0;
            rc = deformed_op(c, 1, &al, &be, y, y, c->Ky);
        } else {
            rc = op(c, c->k, RK_FP64, EPI_STORE, c->form[F_K], y, c->Ky, nullptr, nullptr, c->n, 0, 1, 0, 0);
        }
        if (rc) return rc;
        double c1[RK_MAX_Q], c2[RK_MAX_Q], cf[2 * RK_MAX_Q];
        for (int i = 0; i < Q; ++i) {
            c1[i] = 0.0; c2[i] = 0.0;
            for (int j = 0; j < Q; ++j) {
                c1[i] += c->tab.Ainv[i * Q + j] * (G ? gamma[j] : 0.0);
                c2[i] -= c->tab.Ainv[i * Q + j];
            }
        }
        for (int i = 0; i < Q; ++i) {
            if (!c->cplx) { cf[i] = c1[i]; cf[RK_MAX_Q + i] = c2[i]; continue; }
            double a = 0.0, b = 0.0;
            for (int j = 0; j < Q; ++j) { a += c->tab.CT[i * Q + j] * c1[j]; b += c->tab.CT[i * Q + j] * c2[j]; }
            cf[i] = a; cf[RK_MAX_Q + i] = b;
        }
        HIPCHK(c, hipMemcpyAsync(c->mix + kMixRhs, cf, sizeof(cf), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));   // cf lives on the host stack
        HIPCHK(c, launch_rhs_mix(G, c->Ky, c->rhs, c->mix + kMixRhs, c->mix + kMixRhs + RK_MAX_Q, Q, c->N, c->stream));
    }
    bool converged = false;
    rc = gmres(c, st, converged);
    if (rc) return rc;
    if (converged) {
        Timer t(c, C_REST);
        // y += tau sum_i b_i k_i with k = (U (x) I) u for the complex method
        double bw[RK_MAX_Q];
        for (int s = 0; s < Q; ++s) {
            if (!c->cplx) { bw[s] = c->tab.b[s]; continue; }
            bw[s] = 0.0;
            for (int i = 0; i < Q; ++i) bw[s] += c->tab.b[i] * c->tab.CU[i * Q + s];
        }
        HIPCHK(c, launch_stage_combine(y, c->kv, bw, c->tau, Q, c->N, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->opt.timing) {
        double tt[C_N] = {0};
        for (size_t i = 0; i < c->pool_used; ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, c->event_pool[i].a, c->event_pool[i].b);
            tt[c->event_pool[i].comp] += ms * 1e-3;
        }
        st.t_rhs = tt[C_RHS]; st.t_vmult = tt[C_VMULT]; st.t_basis = tt[C_BASIS];
        st.t_blocks = tt[C_BLOCKS]; st.t_rest = tt[C_REST];
    }
    if (stats) *stats = st;
    if (!converged) return fail(c, RK_ENOCONV, "GMRES did not reach rtol within max_iter");
    return RK_OK;
}

// Stage-DoFs below which a step costs about as much as a step of this size
// (measured on the 64-problem uneven batch: balancing streams by
// max(stage-DoFs, 8M) beat balancing by stage-DoFs by 5-8%).
constexpr double kLatencyFloor = 8.0 * (1 << 20);

int rk_step_batch(rk_ctx* const* ctx, int count, const double* t_n, double* const* y, const double* const* G,
                  const double* gamma, rk_stats* stats, int* codes, int threads) {
    if (count < 0 || (count > 0 && (!ctx || !t_n || !y))) return fail(nullptr, RK_EINVAL, "bad batch arguments");
    for (int i = 0; i < count; ++i) {
        if (!ctx[i] || !y[i]) return fail(nullptr, RK_EINVAL, "NULL context or vector in the batch");
        if (G && G[i] && !gamma) return fail(nullptr, RK_EINVAL, "gamma is NULL while G is given");
        for (int j = 0; j < i; ++j)
            if (ctx[j] == ctx[i]) return fail(nullptr, RK_EINVAL, "a context appears twice in the batch");
    }
    if (count == 0) return RK_OK;
    int nt = threads > 0 ? threads : count;
    nt = std::max(1, std::min(std::min(nt, count), 16));
    std::vector<int> rc(count, RK_OK);
    // Entries are grouped by their context's stream (contexts that share a
    // stream run on one worker, in input order).  The streams go to the
    // workers largest first, each to the least loaded worker, by an estimated
    // cost per step: the stage-DoFs of each context, but at least
    // kLatencyFloor (below that a step is bound by its launch and
    // synchronisation latency, not by its size).
    std::vector<hipStream_t> streams;
    std::vector<std::vector<int>> members;
    std::vector<double> cost;
    for (int i = 0; i < count; ++i) {
        size_t s = 0;
        while (s < streams.size() && streams[s] != ctx[i]->stream) ++s;
        if (s == streams.size()) { streams.push_back(ctx[i]->stream); members.emplace_back(); cost.push_back(0.0); }
        members[s].push_back(i);
        cost[s] += std::max((double)ctx[i]->N3 * ctx[i]->Q, kLatencyFloor);
    }
    std::vector<int> order(streams.size());
    for (size_t s = 0; s < order.size(); ++s) order[s] = (int)s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<std::vector<int>> plan(nt);
    std::vector<double> load(nt, 0.0);
    for (int s : order) {
        const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[w] += cost[s];
        plan[w].insert(plan[w].end(), members[s].begin(), members[s].end());
    }
    auto work = [&](int w) {
        for (int i : plan[w]) {
            if (hipSetDevice(ctx[i]->device) != hipSuccess) { rc[i] = fail(ctx[i], RK_EHIP, "hipSetDevice failed"); continue; }
            rc[i] = rk_step(ctx[i], t_n[i], y[i], G ? G[i] : nullptr, gamma ? gamma + (size_t)i * RK_MAX_Q : nullptr,
                            stats ? stats + i : nullptr);
        }
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        pool.reserve(nt);
        for (int w = 0; w < nt; ++w) pool.emplace_back(work, w);
        for (auto& t : pool) t.join();
    }
    int first = RK_OK;
    for (int i = 0; i < count; ++i) {
        if (codes) codes[i] = rc[i];
        if (first == RK_OK && rc[i] != RK_OK) first = rc[i];
    }
    return first;
}

// ---------------------------------------------------------------------------
// Deformed-mesh operator (context-free).
// ---------------------------------------------------------------------------
namespace {
int check_deformed(const rk_mesh* mesh, int degree, int dtype) {
    if (!mesh || mesh->n_cells < 1 || degree < 1 || degree > RK_MAX_DEGREE)
        return fail(nullptr, RK_EINVAL, "mesh or degree (1..6) out of range");
    if (mesh->length != 1.0)
        return fail(nullptr, RK_EINVAL, "deformed meshes are defined on the unit cube: mesh length must be 1");
    if ((long long)mesh->n_cells * degree + 1 > 16384)
        return fail(nullptr, RK_EINVAL, "grid too large: need n_cells*degree + 1 <= 16384");
    if (dtype != RK_FP64 && dtype != RK_FP32) return fail(nullptr, RK_EINVAL, "bad dtype");
    return RK_OK;
}
}  // namespace

int rk_deformed_geometry_bytes(const rk_mesh* mesh, int degree, int dtype, size_t* bytes) {
    if (!bytes) return fail(nullptr, RK_EINVAL, "bytes is NULL");
    int rc = check_deformed(mesh, degree, dtype);
    if (rc) return rc;
    *bytes = deformed_geometry_elems(mesh->n_cells, degree) * dsize(dtype);
    return RK_OK;
}

int rk_deformed_geometry(const rk_mesh* mesh, int degree, double eps, int dtype, void* d_geometry,
                         void* hip_stream) {
    int rc = check_deformed(mesh, degree, dtype);
    if (rc) return rc;
    if (!d_geometry) return fail(nullptr, RK_EINVAL, "geometry is NULL");
    if (!(std::fabs(eps) <= RK_MAX_DEFORM)) return fail(nullptr, RK_EINVAL, "|eps| must be <= RK_MAX_DEFORM");
    hipError_t e = launch_deformed_geometry(degree, dtype, mesh->n_cells, eps, d_geometry, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, RK_EHIP, std::string("deformed geometry: ") + hipGetErrorString(e));
    return RK_OK;
}

int rk_deformed_apply(const rk_mesh* mesh, int degree, int Q, const double* alpha, const double* beta, int dtype,
                      const void* d_geometry, const void* d_u, void* d_v, void* hip_stream) {
    int rc = check_deformed(mesh, degree, dtype);
    if (rc) return rc;
    if (Q < 1 || Q > RK_MAX_Q) return fail(nullptr, RK_EINVAL, "Q out of range (1..9)");
    if (!alpha || !beta || !d_geometry || !d_u || !d_v) return fail(nullptr, RK_EINVAL, "NULL argument");
    const long long N = (long long)mesh->n_cells * degree + 1;
    const size_t bytes = dsize(dtype) * (size_t)Q * N * N * N;
    if ((const char*)d_u < (const char*)d_v + bytes && (const char*)d_v < (const char*)d_u + bytes)
        return fail(nullptr, RK_EINVAL, "u and v overlap");
    hipError_t e = launch_deformed_apply(degree, dtype, mesh->n_cells, Q, alpha, beta, d_geometry, d_u, d_u, d_v,
                                         (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, RK_EHIP, std::string("deformed apply: ") + hipGetErrorString(e));
    return RK_OK;
}

const char* rk_last_error(const rk_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
