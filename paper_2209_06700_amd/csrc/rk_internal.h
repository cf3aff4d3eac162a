// Internal declarations shared by the host driver and the HIP kernel units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rk.h"

namespace rk {

// ---------------------------------------------------------------------------
// Host-side mathematics (long double; rounded to double for the device).
// ---------------------------------------------------------------------------

// Radau IIA tableau and the factors of the preconditioner of eq. (irk:P).
struct Tableau {
    int Q = 0;
    double A[RK_MAX_Q * RK_MAX_Q], b[RK_MAX_Q], c[RK_MAX_Q];
    double Ainv[RK_MAX_Q * RK_MAX_Q];
    double L[RK_MAX_Q * RK_MAX_Q], U[RK_MAX_Q * RK_MAX_Q];
    double S[RK_MAX_Q * RK_MAX_Q], Sinv[RK_MAX_Q * RK_MAX_Q];
    double lam[RK_MAX_Q];
    // Direct diagonalisation A^-1 = S Lam S^-1 with complex S, Lam (eq.
    // irk:Ainv) in real slot form: nb = ceil(Q/2) blocks, the npair
    // conjugate pairs (one member each, Im > 0, ascending Re) then the real
    // eigenvalue (odd Q).  Slots 0..nb-1 hold the real parts (and the real
    // block), slots nb..Q-1 the imaginary parts, so pair j owns slots j and
    // nb + j.  slots = (CT (x) I) k, k = (CU (x) I) slots, and
    // CT A^-1 CU = CLam with [[a, -b], [b, a]] per pair lam = a + i b.
    int nb = 0, npair = 0;
    double clam_re[RK_MAX_Q], clam_im[RK_MAX_Q];
    double CT[RK_MAX_Q * RK_MAX_Q], CU[RK_MAX_Q * RK_MAX_Q], CLam[RK_MAX_Q * RK_MAX_Q];
    double hshift[RK_MAX_Q];   // per slot: a + b for a pair's slots, lam for the real block
};
// Returns false (with a message) if a factorisation breaks down.
bool build_tableau(int Q, Tableau& t, std::string& err);

// 1D reference element of degree k on [0,1] (Gauss-Lobatto nodes).
struct Element1D {
    int k = 0;
    double nodes[RK_MAX_DEGREE + 1];
    double mass[(RK_MAX_DEGREE + 1) * (RK_MAX_DEGREE + 1)];    // int l_a l_b
    double stiff[(RK_MAX_DEGREE + 1) * (RK_MAX_DEGREE + 1)];   // int l_a' l_b'
    // prolongation from one coarse cell to its two halves: (2k+1) x (k+1)
    double prol[(2 * RK_MAX_DEGREE + 1) * (RK_MAX_DEGREE + 1)];
};
void build_element(int k, Element1D& e);

// Per-stage scales of the diagonal-mix operator v_s = alpha_s Mref u_s +
// beta_s Kref u_s, where Mref / Kref are the Kronecker products of the unit-cell
// 1D element matrices and the cell size is folded into the scales (h^3 for the
// mass term, h for the stiffness term).
struct StageScal {
    double alpha[RK_MAX_Q] = {};
    double beta[RK_MAX_Q] = {};
};

// Independent systems inside one Krylov vector.  Group g (the unknowns of
// one block) is the union of the vector segments q = first[g] .. first[g+1]-1,
// segment q covering elements [off[q], off[q] + len[q]).  The Crout solve
// has one group of one segment (the whole vector); the complex solve has one
// group per block and one segment per slot.
struct Segs {
    int ngroup = 1;
    int first[RK_MAX_Q + 1] = {0, 1};
    long long off[RK_MAX_Q] = {};
    long long len[RK_MAX_Q] = {};
};
// Per-group scalars of Krylov vector i live at [i * kSigStride + g].
constexpr int kSigStride = RK_MAX_Q;
// A slot -> index map (passed by value).
struct SlotIdx {
    int v[RK_MAX_Q] = {};
};

// ---------------------------------------------------------------------------
// Kernel launchers (implemented in the .hip units).  All return hipError_t.
// ---------------------------------------------------------------------------
enum Mix { MIX_DIAG = 0, MIX_PAIR = 1 };
// Epilogues of the operator kernel.  EPI_CHEB1 is EPI_CHEB whose input is
// the first Chebyshev iterate x1 = c0 D^-1 b formed from b while it is staged
// (u = b, x_prev = 0), so x1 is never stored.
enum Epi { EPI_STORE = 0, EPI_RESID = 1, EPI_CHEB = 2, EPI_CHEB1 = 3 };

struct OpLaunch {
    int k = 0;
    int dtype = RK_FP64;
    int mix = MIX_DIAG;
    int epi = EPI_STORE;
    const void* u = nullptr;   // input vector base (stage 0); mass-term input for MIX_PAIR
    const void* u2 = nullptr;  // MIX_PAIR: stiffness-term input base
    void* v = nullptr;         // output vector base (stage 0)
    const void* b = nullptr;   // EPI_RESID / EPI_CHEB right-hand side base
    const void* xo = nullptr;  // EPI_CHEB previous iterate base (nullptr = zero)
    double alpha[RK_MAX_Q] = {};   // per-stage scales: v_s = alpha_s Mref u_s + beta_s Kref u_s
    double beta[RK_MAX_Q] = {};    // (MIX_PAIR: alpha_s Mref u_s + beta_s Kref u2_s)
    long long stride = 0;      // elements between stages (N^3)
    int n = 0;                 // cells per direction
    int s0 = 0, nstage = 1;    // stages [s0, s0 + nstage)
    double ca = 0.0, cb = 0.0; // EPI_CHEB: x_new = x + ca (x - xo) + cb D^-1 (b - A x)
    // EPI_CHEB with xo_from_b: x_prev = c0 D^-1 b (the first iterate, formed
    // from b instead of read); EPI_CHEB1: the input is c0 D^-1 b
    int xo_from_b = 0;
    double c0 = 0.0;
    int cz = 0;                // elements per z-chunk of a work item (0: size heuristic)
    int ts = 0;                // tile shape: 0 (about 32 x-nodes) or 1 (about 64; fp32 diagonal mix)
    hipStream_t stream = nullptr;
};
hipError_t launch_op(const OpLaunch& L);

// Work-list launches of the operator over several problems (contexts) of one
// degree and dtype: the diagonal-mix store form, at most kOpListMax problems
// per launch (their launch descriptors travel in the kernel arguments), on a
// persistent grid of at most kOpListGrid workgroups.
constexpr int kOpListMax = 12;
constexpr int kOpListGrid = 2048;
hipError_t launch_op_list(const OpLaunch* L, int count, hipStream_t stream);

// Records msg as the message of a failed context-free call (rk_last_error(NULL))
// and returns code.
int report_free_error(int code, const std::string& msg);

// Multigrid transfers (one fused pass each).
// coarse = P^T fine for stages [0, nstage): fine grid of 2 nc cells (stage
// stride fstride), coarse grid of nc cells (stride cstride), degree k; coarse
// boundary nodes written as zero.  tmp holds nstage (2 nc k + 1)(nc k + 1)^2
// values (x-y restricted fine planes).
hipError_t launch_restrict(int k, int dtype, const void* fine, void* coarse, void* tmp, int nc, int nstage,
                           long long fstride, long long cstride, hipStream_t st);
// fine += P coarse for stages [0, nstage): coarse grid of nc cells (stage
// stride cstride), fine grid of 2 nc cells (stride fstride), degree k; one pass
hipError_t launch_prolong_add(int k, int dtype, const void* coarse, void* fine, int nc, int nstage,
                              long long cstride, long long fstride, hipStream_t st);

// The coarse end of a V-cycle in one launch (one workgroup per stage block):
// levels lv[0..nlev) are consecutive multigrid levels, lv[0] the finest of
// them.  Per level: the rhs b and the two iterate buffers x ("first") and y
// ("second"), stage-0 bases of [Q][N3] vectors; the block scales
// alpha_s Mref + beta_s Kref; the Chebyshev interval (theta, delta, sigma as
// in the multi-launch path) and degree (the coarse degree on the last level).
// On return the V-cycle result for lv[0].b is in lv[0].y if nlev > 1, else in
// lv[0].x for an odd degree and lv[0].y for an even one.  scratch: per stage
// sstride >= 4 n3max values, n3max >= lv[0].N3.
constexpr int kTailMaxLevels = 8;
struct TailLevel {
    void* b = nullptr;
    void* x = nullptr;
    void* y = nullptr;
    long long N3 = 0;
    int n = 0, degree = 1;
    double theta = 1.0, delta = 1.0, sigma = 1.0;
    double alpha[RK_MAX_Q] = {}, beta[RK_MAX_Q] = {};
};
struct TailArgs {
    TailLevel lv[kTailMaxLevels];
    int nlev = 0, s0 = 0, dtype = RK_FP32;
    void* scratch = nullptr;
    long long sstride = 0, n3max = 0;
};
hipError_t launch_tail_vcycle(int k, const TailArgs& a, int nblocks, hipStream_t st);

// x = cb D^-1 b (first Chebyshev step from a zero start), D = diag of the
// diagonal-mix operator with scales sc, per stage; boundary entries 0.
hipError_t launch_cheb_first(int k, int dtype, const StageScal& sc, const void* b, void* x,
                             int n, int s0, int nstage, double cb, hipStream_t st);

// out_i = sum_j D[i][j] in_j (D: device doubles, row-major Qout x Qin),
// computed in double; in/out dtypes independent.  Boundary entries 0.  If out2
// is not null, out2_i = sum_j D2[i][j] in_j (fp64) is written in the same pass.
// If in_scale (device doubles) is not null, input slot j is multiplied by
// in_scale[scale_idx->v[j]] first (scale_idx null: in_scale[0] for all).
hipError_t launch_stage_mix(int dtype_in, const void* in, int dtype_out, void* out,
                            const double* D, int qout, int qin, int N, hipStream_t st,
                            double* out2 = nullptr, const double* D2 = nullptr,
                            const double* in_scale = nullptr, const SlotIdx* scale_idx = nullptr);

// out_i = c1[i] G + c2[i] w on interior nodes, 0 on boundary nodes (fp64, N
// nodes per direction); G may be null.  c1, c2: device doubles.
hipError_t launch_rhs_mix(const double* G, const double* w, double* out, const double* c1,
                          const double* c2, int Q, int N, hipStream_t st);

// Partial dot products per group g of sg (workgroup blk of nblocks):
// part[(g nblocks + blk) nout + l] = sum over the group's entries in blk of
// X_l[i] w[i] for l < nvec, and (if self) at l = nvec of w[i]^2;
// nout = nvec + self.
hipError_t launch_dots(const double* X, int nvec, long long ld, const double* w, const Segs& sg,
                       int self, double* part, int nblocks, hipStream_t st);
// Per group g: out = w - sum_l h[g hstride + l] sig[l kSigStride + g] X_l
// (sig may be null = ones; out may alias w); if norm_part:
// norm_part[g nblocks + blk] = sum of out^2 over the group's entries in blk.
hipError_t launch_gs_update(const double* X, int nvec, long long ld, const double* h, int hstride,
                            const double* sig, const double* w, double* out, const Segs& sg,
                            double* norm_part, int nblocks, hipStream_t st);
// For g < ngroup and l < nout: out[g ostride + l] (+)= scale[l kSigStride + g]
// * sum_b part[(g nblocks + b) nout + l] (fixed order; scale applies to
// l < nscale).  If inv_sqrt_out: inv_sqrt_out[g] = 1/sqrt(out[g ostride + nout-1]).
hipError_t launch_reduce(const double* part, int nblocks, int nout, double* out, int accumulate,
                         hipStream_t st, const double* scale = nullptr, int nscale = 0,
                         double* inv_sqrt_out = nullptr, int ngroup = 1, int ostride = 0);
// Per group g: k += sum_j y[g ystride + j] Z_j over the group's entries
// (Z fp64 or fp32)
hipError_t launch_combine(double* kv, int dtype_z, const void* Z, int nz, long long ld,
                          const double* y, int ystride, const Segs& sg, hipStream_t st);
// y += tau sum_i b[i] k_i on interior nodes, y = 0 on boundary nodes
// (b: host values, passed by value; N nodes per direction)
hipError_t launch_stage_combine(double* y, const double* kv, const double* b, double tau, int Q,
                                int N, hipStream_t st);
hipError_t launch_fill(int dtype, void* x, long long n, double value, hipStream_t st);
hipError_t launch_copy(int dtype, const void* src, void* dst, long long n, hipStream_t st);
// v = b - v (fp64)
hipError_t launch_sub_from(double* v, const double* b, long long n, hipStream_t st);

// Deformed-mesh operator (deformed_kernels.hip).  Geometry: per cell and
// Gauss point the 7 values m = w det J, G = w det J J^-1 J^-T (xx, yy, zz, xy,
// xz, yz) for the map x + eps sin(pi x1) sin(pi x2) sin(pi x3) (1,1,1),
// stored [cell][7][point] (cells x fastest, points x fastest); element count
// from deformed_geometry_elems.  Apply: v_s = alpha_s M u_s + beta_s K u_s for
// s < Q on [Q][N^3] vectors (boundary entries read as 0, written 0); v is
// overwritten.  With um != u the mass term takes um: v_s = alpha_s M um_s +
// beta_s K u_s.  alpha, beta: host arrays of Q values.
size_t deformed_geometry_elems(int n, int k);
hipError_t launch_deformed_geometry(int k, int dtype, int n, double eps, void* geo, hipStream_t st);
hipError_t launch_deformed_apply(int k, int dtype, int n, int Q, const double* alpha, const double* beta,
                                 const void* geo, const void* um, const void* u, void* v, hipStream_t st);
// Jacobi diagonals of the deformed-mesh M and K into dM, dK ([N^3], dtype).
hipError_t launch_deformed_diag(int k, int dtype, int n, const void* geo, void* dM, void* dK, hipStream_t st);
// x_new = x + ca (x - xo) + cb D^-1 (b - t), D_s = alpha_s dM + beta_s dK, on
// interior nodes of nstage stages (x, xo, t may be null = 0; x_new may alias
// x or xo), boundary 0.  alpha, beta: host arrays of nstage values.
hipError_t launch_cheb_vec(int dtype, void* xn, const void* x, const void* xo, const void* b, const void* t,
                           const void* dM, const void* dK, const double* alpha, const double* beta, double ca,
                           double cb, int N, int nstage, hipStream_t st);
// v = b - v, n entries of dtype
hipError_t launch_resid_vec(int dtype, void* v, const void* b, long long n, hipStream_t st);

// Power iteration support (per stage, diagonal-mix operator with scales sc):
// given v and w = A v: z = D^-1 w; part[blk*3*ns + 3 s + {0,1,2}] =
// {v.w, v.Dv, z.z} restricted to stage s.  Requires nstage <= RK_MAX_Q.  With
// dMv, dKv (stored [N^3] diagonals) D_s = alpha_s dMv + beta_s dKv, else the
// affine-mesh diagonal from the 1D tables.
hipError_t launch_power_partial(int k, int dtype, const StageScal& sc, const void* v,
                                const void* w, void* z, int n, int nstage, double* part,
                                int nblocks, hipStream_t st, const void* dMv = nullptr,
                                const void* dKv = nullptr);
// v_s = z_s / sqrt(zz_s) with zz_s = red[3 s + 2]
hipError_t launch_power_normalize(int dtype, const void* z, void* v, const double* red, int n,
                                  int nstage, hipStream_t st);
// deterministic pseudo-random start vector in [-1,1], zero boundary
hipError_t launch_random_fill(int dtype, void* x, int N, int nstage, unsigned seed,
                              hipStream_t st);

}  // namespace rk
