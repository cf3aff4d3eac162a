// rk_apply_operator_static: the operator forms of rk_apply_operator for a
// mesh, degree, stage count and tau given per call, with no context, no
// workspace and no allocation.  The dense forms mix the input stages first;
// that mixed input and the Q x Q mixing table live in `scratch`, a file-scope
// device array of fixed size that every GPU the library runs on holds until
// the process ends.
//
// Host code never passes the array's name to a kernel: in host code it is a
// stand-in, not a device address.  The address is fetched once per device
// with hipGetSymbolAddress (with that device current) and kept in
// g_scratch[device]; kernels and copies take that pointer.
//
// All calls on one GPU share its array and it keeps the last call's contents.
// Every byte a call reads is written earlier in the same call (the table by
// put_table, the mixed input by the stage mix), so nothing has to be cleared.
// Calls that overlap in time on one GPU race on the array.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "rk_internal.h"

namespace rk {
namespace {

constexpr size_t kTableBytes = 4096;                          // Q x Q doubles, Q <= 9
constexpr size_t kMixBytes = RK_STATIC_SCRATCH_BYTES;         // mixed input stages
static __device__ __align__(256) unsigned char scratch[kTableBytes + kMixBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
Tableau g_tab[RK_MAX_Q + 1];
bool g_tab_ok[RK_MAX_Q + 1] = {};

// Device address of this GPU's array (set up on the first call per device).
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_free_error(RK_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return report_free_error(RK_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return report_free_error(RK_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return RK_OK;
}

// Radau IIA tableau of Q stages (host, cached per Q).
int tableau(int Q, const Tableau** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tab_ok[Q]) {
        std::string msg;
        if (!build_tableau(Q, g_tab[Q], msg)) return report_free_error(RK_EINVAL, msg);
        g_tab_ok[Q] = true;
    }
    *out = &g_tab[Q];
    return RK_OK;
}

struct MixTable {
    double d[RK_MAX_Q * RK_MAX_Q];
};

// dst[i] = t.d[i] for i < count (the table travels as a kernel argument: no
// host-to-device copy).
__global__ void put_table(double* dst, MixTable t, int count) {
    const int i = threadIdx.x;
    if (i < count) dst[i] = t.d[i];
}

}  // namespace
}  // namespace rk

extern "C" int rk_apply_operator_static(const rk_mesh* mesh, int degree, int Q, double tau, int form, int dtype,
                                        const void* d_u, void* d_v, void* hip_stream) {
    using namespace rk;
    if (!mesh || mesh->n_cells < 1 || degree < 1 || degree > RK_MAX_DEGREE)
        return report_free_error(RK_EINVAL, "mesh or degree (1..6) out of range");
    if (!(mesh->length > 0.0) || !std::isfinite(mesh->length))
        return report_free_error(RK_EINVAL, "mesh length must be finite and > 0");
    if ((long long)mesh->n_cells * degree + 1 > 16384)
        return report_free_error(RK_EINVAL, "grid too large: need n_cells*degree + 1 <= 16384");
    if (Q < 1 || Q > RK_MAX_Q) return report_free_error(RK_EINVAL, "Q out of range (1..9)");
    if (!(tau > 0.0)) return report_free_error(RK_EINVAL, "tau must be > 0");
    if (form != RK_OP_CALA && form != RK_OP_STAGE && form != RK_OP_BLOCKS && form != RK_OP_K && form != RK_OP_M)
        return report_free_error(RK_EINVAL, "bad operator form (CALA, STAGE, BLOCKS, K or M)");
    if (dtype != RK_FP64 && dtype != RK_FP32) return report_free_error(RK_EINVAL, "bad dtype");
    if (!d_u || !d_v) return report_free_error(RK_EINVAL, "NULL vector");
    const int n = mesh->n_cells;
    const long long N = (long long)n * degree + 1, N3 = N * N * N;
    const int ns = (form == RK_OP_K || form == RK_OP_M) ? 1 : Q;
    const size_t esz = dtype == RK_FP64 ? 8 : 4;
    const size_t bytes = esz * (size_t)ns * (size_t)N3;
    if ((const char*)d_u < (const char*)d_v + bytes && (const char*)d_v < (const char*)d_u + bytes)
        return report_free_error(RK_EINVAL, "u and v overlap");
    const bool pair = form == RK_OP_CALA || form == RK_OP_STAGE;
    if (pair && bytes > kMixBytes)
        return report_free_error(RK_EINVAL, "Q N^3 values exceed the static scratch of rk_apply_operator_static (" +
                                                std::to_string(kMixBytes >> 20) + " MiB)");
    const Tableau* tab = nullptr;
    int rc = tableau(Q, &tab);
    if (rc) return rc;

    // v_s = alpha_s Mref uM_s + beta_s Kref uK_s with the cell size folded in
    // (h^3 for the mass term, h for the stiffness term), as in the context.
    const double h = mesh->length / n, h3 = h * h * h;
    OpLaunch L;
    L.k = degree;
    L.dtype = dtype;
    L.mix = pair ? MIX_PAIR : MIX_DIAG;
    L.epi = EPI_STORE;
    L.stride = N3;
    L.n = n;
    L.s0 = 0;
    L.nstage = ns;
    L.stream = (hipStream_t)hip_stream;
    for (int s = 0; s < RK_MAX_Q; ++s) {
        L.alpha[s] = form == RK_OP_BLOCKS ? (s < Q ? tab->lam[s] * h3 : 0.0) : form == RK_OP_K ? 0.0 : h3;
        L.beta[s] = form == RK_OP_M ? 0.0 : form == RK_OP_K ? h : tau * h;
    }
    L.u = d_u;
    L.v = d_v;
    hipError_t e;
    if (pair) {
        void* base = nullptr;
        rc = scratch_address(&base);
        if (rc) return rc;
        double* table = static_cast<double*>(base);
        void* mixed = static_cast<unsigned char*>(base) + kTableBytes;
        // CALA: the mass term takes (A^-1 (x) I) u (eq. irk:A); STAGE: the
        // stiffness term takes (A (x) I) u (the stage system of Sec. 2)
        MixTable t{};
        std::memcpy(t.d, form == RK_OP_CALA ? tab->Ainv : tab->A, sizeof(double) * Q * Q);
        put_table<<<1, 128, 0, L.stream>>>(table, t, Q * Q);
        e = hipGetLastError();
        if (e != hipSuccess) return report_free_error(RK_EHIP, std::string("put_table: ") + hipGetErrorString(e));
        e = launch_stage_mix(dtype, d_u, dtype, mixed, table, Q, Q, (int)N, L.stream);
        if (e != hipSuccess) return report_free_error(RK_EHIP, std::string("stage mix: ") + hipGetErrorString(e));
        L.u = form == RK_OP_CALA ? mixed : d_u;
        L.u2 = form == RK_OP_CALA ? d_u : mixed;
    }
    e = launch_op(L);
    if (e != hipSuccess) return report_free_error(RK_EHIP, std::string("operator: ") + hipGetErrorString(e));
    return RK_OK;
}
