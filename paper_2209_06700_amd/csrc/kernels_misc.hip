// Streaming kernels: Chebyshev start, stage mixes (basis changes, right-hand
// side), Krylov vector operations, reductions and the stage combination.  All
// are bandwidth-bound with coalesced x-fastest access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <utility>

#include "element_data.h"
#include "rk_internal.h"

namespace rk {
namespace {

constexpr int kBlock = 256;
constexpr int kMP = RK_MAX_DEGREE + 1;

// Element tables of every degree for kernels that index them at run time.
struct AllTables {
    double dM[kMP][kMP];                            // 1D global mass diagonal by local index
    double dA[kMP][kMP];                            // 1D global stiffness diagonal by local index
};

template <int K>
constexpr void fill_tables(AllTables& t) {
    constexpr auto d = elem::make<K>();
    for (int r = 0; r < K; ++r) {
        t.dM[K][r] = r == 0 ? d.M[0][0] + d.M[K][K] : d.M[r][r];
        t.dA[K][r] = r == 0 ? d.A[0][0] + d.A[K][K] : d.A[r][r];
    }
}

constexpr AllTables make_tables() {
    AllTables t{};
    fill_tables<1>(t);
    fill_tables<2>(t);
    fill_tables<3>(t);
    fill_tables<4>(t);
    fill_tables<5>(t);
    fill_tables<6>(t);
    return t;
}

__constant__ AllTables kTab = make_tables();

template <typename T>
struct Scal {
    T alpha[RK_MAX_Q], beta[RK_MAX_Q];
};

template <typename T>
Scal<T> to_scal(const StageScal& s) {
    Scal<T> o;
    for (int i = 0; i < RK_MAX_Q; ++i) { o.alpha[i] = T(s.alpha[i]); o.beta[i] = T(s.beta[i]); }
    return o;
}

inline int grid_for(long long n, int cap = 8192) {
    long long g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

// ---------------------------------------------------------------------------
// Jacobi diagonal of the diagonal-mix operator (scales alpha, beta) at node
// (x, y, z) of a degree-k grid.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T jacobi_diag(int k, T alpha, T beta, int x, int y, int z) {
    const T mx = T(kTab.dM[k][x % k]), my = T(kTab.dM[k][y % k]), mz = T(kTab.dM[k][z % k]);
    const T kx = T(kTab.dA[k][x % k]), ky = T(kTab.dA[k][y % k]), kz = T(kTab.dA[k][z % k]);
    return fma(alpha, mx * my * mz, beta * (kx * my * mz + mx * ky * mz + mx * my * kz));
}

// 1/d; fp32 takes the hardware reciprocal (the smoother is a preconditioner)
template <typename T>
__device__ __forceinline__ T smoother_recip(T d) {
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(d);
    else return T(1) / d;
}

// First Chebyshev iterate from a zero guess: x = cb D^-1 b on interior nodes,
// 0 on the boundary.  Block (64, 4) covers four node rows; grid (ceil(N / 4),
// N * nstage) gives every block one (stage, z) plane slice, so no thread
// divides a flat index.
constexpr int kRowThreads = 64, kRows = kBlock / kRowThreads;

template <typename T>
__global__ void __launch_bounds__(kBlock) cheb_first_kernel(Scal<T> sc, int k,
                                                            const T* __restrict__ b, T* __restrict__ x,
                                                            int n, int s0, T cb) {
    const int nK = n * k, N = nK + 1;
    const int y = blockIdx.x * kRows + threadIdx.y;
    const int sl = blockIdx.y / N, z = blockIdx.y - sl * N;
    if (y >= N) return;
    const int s = s0 + sl;
    const long long row = (long long)s * N * N * N + ((long long)z * N + y) * N;
    const bool yz_in = y > 0 && y < nK && z > 0 && z < nK;
    const int ry = y % k, rz = z % k;
    const T my = T(kTab.dM[k][ry]), mz = T(kTab.dM[k][rz]);
    const T ky = T(kTab.dA[k][ry]), kz = T(kTab.dA[k][rz]);
    const T myz = my * mz, kyz = ky * mz + my * kz;
    const T al = sc.alpha[s], be = sc.beta[s];
    const int step = kRowThreads % k;
    int r = threadIdx.x % k;
    for (int xx = threadIdx.x; xx < N; xx += kRowThreads) {
        T val = T(0);
        if (yz_in && xx > 0 && xx < nK) {
            const T mx = T(kTab.dM[k][r]), kx = T(kTab.dA[k][r]);
            const T D = fma(al, mx * myz, be * fma(kx, myz, mx * kyz));
            val = cb * b[row + xx] * smoother_recip(D);
        }
        x[row + xx] = val;
        r += step;
        if (r >= k) r -= k;
    }
}

// ---------------------------------------------------------------------------
// Stage mixes.
// ---------------------------------------------------------------------------
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) stage_mix_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                           const double* __restrict__ D, int qout,
                                                           int qin, int N, double* __restrict__ out2,
                                                           const double* __restrict__ D2,
                                                           const double* __restrict__ in_scale,
                                                           SlotIdx sidx) {
    double isc[RK_MAX_Q];
#pragma unroll
    for (int j = 0; j < RK_MAX_Q; ++j) isc[j] = (in_scale && j < qin) ? in_scale[sidx.v[j]] : 1.0;
    const int nK = N - 1;
    const long long N3 = (long long)N * N * N;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N3;
         r += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(r / ((long long)N * N));
        const int rr = (int)(r - (long long)z * N * N);
        const int y = rr / N, x = rr - y * N;
        const bool inner = x > 0 && x < nK && y > 0 && y < nK && z > 0 && z < nK;
        double u[RK_MAX_Q];
#pragma unroll
        for (int j = 0; j < RK_MAX_Q; ++j) u[j] = (j < qin && inner) ? isc[j] * (double)in[(long long)j * N3 + r] : 0.0;
#pragma unroll
        for (int i = 0; i < RK_MAX_Q; ++i) {
            if (i >= qout) break;
            double acc = 0.0, acc2 = 0.0;
#pragma unroll
            for (int j = 0; j < RK_MAX_Q; ++j)
                if (j < qin) {
                    acc = fma(D[i * qin + j], u[j], acc);
                    if (out2) acc2 = fma(D2[i * qin + j], u[j], acc2);
                }
            out[(long long)i * N3 + r] = (Tout)acc;
            if (out2) out2[(long long)i * N3 + r] = acc2;
        }
    }
}

// The same mix for qin = qout = Q known at compile time: the coefficients
// stay in registers, one thread per node, the plane index from the grid's y
// dimension and 32-bit in-plane indexing (N^2 < 2^31).
template <typename Tin, typename Tout, int Q, bool TWO>
__global__ void __launch_bounds__(kBlock) stage_mix_q_kernel(const Tin* __restrict__ in, Tout* __restrict__ out,
                                                             const double* __restrict__ D, int N,
                                                             double* __restrict__ out2,
                                                             const double* __restrict__ D2,
                                                             const double* __restrict__ in_scale,
                                                             SlotIdx sidx) {
    const int z = blockIdx.y;
    const unsigned NN = (unsigned)N * (unsigned)N;
    const unsigned t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= NN) return;
    const unsigned y = t / (unsigned)N, x = t - y * (unsigned)N;
    const int nK = N - 1;
    const bool inner = x > 0 && (int)x < nK && y > 0 && (int)y < nK && z > 0 && z < nK;
    const long long N3 = (long long)NN * N;
    const long long r = (long long)z * NN + t;
    double u[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const double sc = in_scale ? in_scale[sidx.v[j]] : 1.0;
        u[j] = inner ? sc * (double)in[(long long)j * N3 + r] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double acc = 0.0, acc2 = 0.0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            acc = fma(D[i * Q + j], u[j], acc);
            if (TWO) acc2 = fma(D2[i * Q + j], u[j], acc2);
        }
        out[(long long)i * N3 + r] = (Tout)acc;
        if (TWO) out2[(long long)i * N3 + r] = acc2;
    }
}

// out_i = c1_i G + c2_i w on interior nodes, 0 on boundary nodes (the load
// vector's boundary entries belong to eliminated Dirichlet unknowns).
__global__ void __launch_bounds__(kBlock) rhs_mix_kernel(const double* __restrict__ G, const double* __restrict__ w,
                                                         double* __restrict__ out,
                                                         const double* __restrict__ c1,
                                                         const double* __restrict__ c2, int Q, int N) {
    const long long n3 = (long long)N * N * N;
    const int nK = N - 1;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n3;
         r += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(r / ((long long)N * N));
        const int rr = (int)(r - (long long)z * N * N);
        const int y = rr / N, x = rr - y * N;
        const bool inner = x > 0 && x < nK && y > 0 && y < nK && z > 0 && z < nK;
        const double g = (G && inner) ? G[r] : 0.0;
        const double wv = inner ? w[r] : 0.0;
        for (int i = 0; i < Q; ++i) out[(long long)i * n3 + r] = fma(c1[i], g, c2[i] * wv);
    }
}

// ---------------------------------------------------------------------------
// Reductions: wave64 shuffles, then LDS across the block's waves, then a
// second fixed-order pass over the per-block partial sums (deterministic).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;   // valid in thread 0
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  Each launch handles a chunk of NV <= 16 basis
// vectors (compile time, so every load of an iteration is issued before the
// arithmetic that uses it); with V2 every thread moves two consecutive
// entries per vector (16-byte loads; needs 16-byte aligned vectors and an even
// leading dimension).  Sums run over a fixed grid with a fixed per-thread
// order, so results are reproducible run to run.
// ---------------------------------------------------------------------------
constexpr int kChunk = 16;

template <typename F, int... I>
hipError_t dispatch_nv_impl(int nv, F&& f, std::integer_sequence<int, I...>) {
    hipError_t e = hipErrorInvalidValue;
    ((nv == I + 1 ? (e = f(std::integral_constant<int, I + 1>{}), 0) : 0), ...);
    return e;
}
// f(integral_constant<int, nv>) for nv in 1..kChunk
template <typename F>
hipError_t dispatch_nv(int nv, F&& f) {
    return dispatch_nv_impl(nv, f, std::make_integer_sequence<int, kChunk>{});
}

template <typename T>
struct Pair;
template <>
struct Pair<double> { using type = double2; };
template <>
struct Pair<float> { using type = float2; };

// Segment loop helper: calls f2(i) for the 16-byte aligned pairs (i, i+1) of
// the segment [o, o + n) that fall to this thread (grid-stride), and f1(i)
// on thread 0 for the unpaired head (odd o) and tail elements.
template <bool V2, typename F2, typename F1>
__device__ __forceinline__ void seg_loop(long long o, long long n, long long tid, long long step, F2&& f2,
                                         F1&& f1) {
    if constexpr (V2) {
        if ((o & 1) && n > 0) {
            if (tid == 0) f1(o);
            ++o;
            --n;
        }
        const long long n2 = n >> 1;
        for (long long i = tid; i < n2; i += step) f2(o + 2 * i);
        if ((n & 1) && tid == 0) f1(o + n - 1);
    } else {
        for (long long i = tid; i < n; i += step) f1(o + i);
    }
}

// For every group g of the segments:
//   part[(g * gridDim.x + blk) * nout + l0 + u] = sum over the block's entries
//   of group g of X_u[i] w[i] (u < NV), and if self the same at l0 + NV for
//   sum w[i]^2.
template <int NV, bool V2>
__global__ void __launch_bounds__(kBlock) dots_kernel(const double* __restrict__ X, long long ld,
                                                      const double* __restrict__ w, Segs sg, int self,
                                                      double* __restrict__ part, int nout, int l0) {
    __shared__ double sh[kBlock / 64];
    constexpr int NA = NV > 0 ? NV : 1;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long step = (long long)gridDim.x * blockDim.x;
    for (int g = 0; g < sg.ngroup; ++g) {
        double acc[NA], accs = 0.0;
#pragma unroll
        for (int u = 0; u < NA; ++u) acc[u] = 0.0;
        auto pair = [&](long long i) {
            const double2 wi = *reinterpret_cast<const double2*>(w + i);
            double2 xv[NA];
#pragma unroll
            for (int u = 0; u < NV; ++u) xv[u] = *reinterpret_cast<const double2*>(X + u * ld + i);
#pragma unroll
            for (int u = 0; u < NV; ++u) acc[u] = fma(xv[u].y, wi.y, fma(xv[u].x, wi.x, acc[u]));
            accs = fma(wi.y, wi.y, fma(wi.x, wi.x, accs));
        };
        auto one = [&](long long i) {
            const double wi = w[i];
            double xv[NA];
#pragma unroll
            for (int u = 0; u < NV; ++u) xv[u] = X[u * ld + i];
#pragma unroll
            for (int u = 0; u < NV; ++u) acc[u] = fma(xv[u], wi, acc[u]);
            accs = fma(wi, wi, accs);
        };
        for (int q = sg.first[g]; q < sg.first[g + 1]; ++q) seg_loop<V2>(sg.off[q], sg.len[q], tid, step, pair, one);
        double* pg = part + ((long long)g * gridDim.x + blockIdx.x) * nout + l0;
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const double t = block_sum(acc[u], sh);
            if (threadIdx.x == 0) pg[u] = t;
        }
        if (self) {
            const double t = block_sum(accs, sh);
            if (threadIdx.x == 0) pg[NV] = t;
        }
    }
}

// Per group g: out = src - sum_u h[g hstride + u] sig[u kSigStride + g] X_u
// over the group's segments (sig may be null; out may alias src); if
// norm_part: norm_part[g gridDim.x + blk] = sum of out^2 over the block's
// entries of the group.
template <int NV, bool V2>
__global__ void __launch_bounds__(kBlock) gs_update_kernel(const double* __restrict__ X, long long ld,
                                                           const double* __restrict__ h, int hstride,
                                                           const double* __restrict__ sig,
                                                           const double* src, double* out, Segs sg,
                                                           double* __restrict__ norm_part) {
    __shared__ double sh[kBlock / 64];
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long step = (long long)gridDim.x * blockDim.x;
    for (int g = 0; g < sg.ngroup; ++g) {
        double coef[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) coef[u] = -h[g * hstride + u] * (sig ? sig[u * kSigStride + g] : 1.0);
        double nrm = 0.0;
        auto pair = [&](long long i) {
            double2 acc = *reinterpret_cast<const double2*>(src + i);
            double2 xv[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) xv[u] = *reinterpret_cast<const double2*>(X + u * ld + i);
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                acc.x = fma(coef[u], xv[u].x, acc.x);
                acc.y = fma(coef[u], xv[u].y, acc.y);
            }
            *reinterpret_cast<double2*>(out + i) = acc;
            nrm = fma(acc.y, acc.y, fma(acc.x, acc.x, nrm));
        };
        auto one = [&](long long i) {
            double acc = src[i];
            double xv[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) xv[u] = X[u * ld + i];
#pragma unroll
            for (int u = 0; u < NV; ++u) acc = fma(coef[u], xv[u], acc);
            out[i] = acc;
            nrm = fma(acc, acc, nrm);
        };
        for (int q = sg.first[g]; q < sg.first[g + 1]; ++q) seg_loop<V2>(sg.off[q], sg.len[q], tid, step, pair, one);
        if (norm_part) {
            const double t = block_sum(nrm, sh);
            if (threadIdx.x == 0) norm_part[(long long)g * gridDim.x + blockIdx.x] = t;
        }
    }
}

// Block (l, g): out[g ostride + l] (+)= scale[l kSigStride + g] * sum_b
// part[(g nblocks + b) nout + l]; for l = nout - 1 also inv_sqrt_out[g].
__global__ void reduce_kernel(const double* __restrict__ part, int nblocks, int nout,
                              double* __restrict__ out, int ostride, int accumulate,
                              const double* __restrict__ scale, int nscale, double* __restrict__ inv_sqrt_out) {
    __shared__ double sh[kBlock / 64];
    const int l = blockIdx.x, g = blockIdx.y;
    const double* pg = part + (long long)g * nblocks * nout;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += pg[(long long)b * nout + l];
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        if (scale && l < nscale) t *= scale[l * kSigStride + g];
        double* o = out + (long long)g * ostride + l;
        *o = accumulate ? *o + t : t;
        if (inv_sqrt_out && l == nout - 1) inv_sqrt_out[g] = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    }
}


// kv += sum_u y[g ystride + u] Z_u over the segments of every group g, for
// a chunk of NV vectors (Z fp64 or fp32)
template <int NV, typename TZ, bool V2>
__global__ void __launch_bounds__(kBlock) combine_kernel(double* __restrict__ kv, const TZ* __restrict__ Z,
                                                         long long ld, const double* __restrict__ y,
                                                         int ystride, Segs sg) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long step = (long long)gridDim.x * blockDim.x;
    for (int g = 0; g < sg.ngroup; ++g) {
        double coef[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) coef[u] = y[g * ystride + u];
        auto pair = [&](long long i) {
            using P2 = typename Pair<TZ>::type;
            double2 acc = *reinterpret_cast<const double2*>(kv + i);
            P2 zv[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) zv[u] = *reinterpret_cast<const P2*>(Z + u * ld + i);
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                acc.x = fma(coef[u], (double)zv[u].x, acc.x);
                acc.y = fma(coef[u], (double)zv[u].y, acc.y);
            }
            *reinterpret_cast<double2*>(kv + i) = acc;
        };
        auto one = [&](long long i) {
            double acc = kv[i];
#pragma unroll
            for (int u = 0; u < NV; ++u) acc = fma(coef[u], (double)Z[u * ld + i], acc);
            kv[i] = acc;
        };
        for (int q = sg.first[g]; q < sg.first[g + 1]; ++q) seg_loop<V2>(sg.off[q], sg.len[q], tid, step, pair, one);
    }
}

struct BVec {
    double v[RK_MAX_Q];
};

// y <- y + tau sum_i b_i k_i on interior nodes; boundary nodes are set to 0.
__global__ void __launch_bounds__(kBlock) stage_combine_kernel(double* __restrict__ y, const double* __restrict__ kv,
                                                               BVec b, double tau, int Q, int N) {
    const long long n3 = (long long)N * N * N;
    const int nK = N - 1;
    for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n3;
         r += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(r / ((long long)N * N));
        const int rr = (int)(r - (long long)z * N * N);
        const int yy = rr / N, x = rr - yy * N;
        double out = 0.0;
        if (x > 0 && x < nK && yy > 0 && yy < nK && z > 0 && z < nK) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < RK_MAX_Q; ++i)
                if (i < Q) acc = fma(b.v[i], kv[(long long)i * n3 + r], acc);
            out = fma(tau, acc, y[r]);
        }
        y[r] = out;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) fill_kernel(T* __restrict__ x, long long n, T value) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = value;
}

// v = b - v
__global__ void __launch_bounds__(kBlock) sub_from_kernel(double* __restrict__ v, const double* __restrict__ b,
                                                          long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        v[i] = b[i] - v[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) copy_kernel(const T* __restrict__ src, T* __restrict__ dst, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Power iteration for the largest eigenvalue of D^-1 A per stage.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) power_partial_kernel(Scal<T> sc, int k,
                                                               const T* __restrict__ v, const T* __restrict__ w,
                                                               T* __restrict__ z, int n, int nstage,
                                                               double* __restrict__ part,
                                                               const T* __restrict__ dMv,
                                                               const T* __restrict__ dKv) {
    __shared__ double sh[kBlock / 64];
    const int nK = n * k, N = nK + 1;
    const long long N3 = (long long)N * N * N;
    for (int s = 0; s < nstage; ++s) {
        double vw = 0.0, vdv = 0.0, zz = 0.0;
        for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < N3;
             r += (long long)gridDim.x * blockDim.x) {
            const int zc = (int)(r / ((long long)N * N));
            const int rr = (int)(r - (long long)zc * N * N);
            const int y = rr / N, x = rr - y * N;
            const long long off = (long long)s * N3 + r;
            T zv = T(0);
            if (x > 0 && x < nK && y > 0 && y < nK && zc > 0 && zc < nK) {
                const double D = dMv ? (double)sc.alpha[s] * (double)dMv[r] + (double)sc.beta[s] * (double)dKv[r]
                                     : (double)jacobi_diag(k, sc.alpha[s], sc.beta[s], x, y, zc);
                const double vv = (double)v[off], wv = (double)w[off];
                vw = fma(vv, wv, vw);
                vdv = fma(vv * D, vv, vdv);
                zv = (T)(wv / D);
                zz = fma((double)zv, (double)zv, zz);
            }
            z[off] = zv;
        }
        double t = block_sum(vw, sh);
        if (threadIdx.x == 0) part[(long long)blockIdx.x * 3 * nstage + 3 * s + 0] = t;
        t = block_sum(vdv, sh);
        if (threadIdx.x == 0) part[(long long)blockIdx.x * 3 * nstage + 3 * s + 1] = t;
        t = block_sum(zz, sh);
        if (threadIdx.x == 0) part[(long long)blockIdx.x * 3 * nstage + 3 * s + 2] = t;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) power_normalize_kernel(const T* __restrict__ z, T* __restrict__ v,
                                                                 const double* __restrict__ red, long long N3,
                                                                 int nstage) {
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N3 * nstage;
         idx += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(idx / N3);
        const double zz = red[3 * s + 2];
        v[idx] = zz > 0.0 ? (T)((double)z[idx] / sqrt(zz)) : T(0);
    }
}

__device__ __forceinline__ unsigned hash32(unsigned x) {
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    return x;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) random_fill_kernel(T* __restrict__ x, int N, int nstage, unsigned seed) {
    const long long N3 = (long long)N * N * N;
    const int nK = N - 1;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N3 * nstage;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long r = idx % N3;
        const int z = (int)(r / ((long long)N * N));
        const int rr = (int)(r - (long long)z * N * N);
        const int y = rr / N, xx = rr - y * N;
        T val = T(0);
        if (xx > 0 && xx < nK && y > 0 && y < nK && z > 0 && z < nK) {
            const unsigned h = hash32((unsigned)idx * 2654435761U ^ seed);
            val = (T)((double)h * (2.0 / 4294967295.0) - 1.0);
        }
        x[idx] = val;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

hipError_t launch_cheb_first(int k, int dtype, const StageScal& sc, const void* b, void* x, int n,
                             int s0, int nstage, double cb, hipStream_t st) {
    const int N = n * k + 1;
    dim3 g((N + kRows - 1) / kRows, N * nstage), blk(kRowThreads, kRows);
    if (dtype == RK_FP64)
        cheb_first_kernel<double><<<g, blk, 0, st>>>(to_scal<double>(sc), k, (const double*)b, (double*)x, n, s0, cb);
    else
        cheb_first_kernel<float><<<g, blk, 0, st>>>(to_scal<float>(sc), k, (const float*)b, (float*)x, n, s0, (float)cb);
    return hipGetLastError();
}

// f(integral_constant<int, q>) for q in 1..RK_MAX_Q
template <typename F>
hipError_t dispatch_q(int q, F&& f) {
    return dispatch_nv_impl(q, f, std::make_integer_sequence<int, RK_MAX_Q>{});
}

hipError_t launch_stage_mix(int dtype_in, const void* in, int dtype_out, void* out, const double* D,
                            int qout, int qin, int N, hipStream_t st, double* out2, const double* D2,
                            const double* in_scale, const SlotIdx* scale_idx) {
    const long long N3 = (long long)N * N * N;
    dim3 g(grid_for(N3)), b(kBlock);
    SlotIdx sidx;
    for (int j = 0; j < RK_MAX_Q; ++j) sidx.v[j] = scale_idx ? scale_idx->v[j] : 0;
    if (qin == qout && (long long)N * N < (1ll << 31) && N <= 65535) {
        const dim3 gq((unsigned)(((long long)N * N + kBlock - 1) / kBlock), (unsigned)N);
        hipError_t e = dispatch_q(qin, [&](auto QC) {
            constexpr int QQ = decltype(QC)::value;
            auto go = [&](auto tin, auto tout) {
                using Ti = decltype(tin);
                using To = decltype(tout);
                if (out2)
                    stage_mix_q_kernel<Ti, To, QQ, true><<<gq, b, 0, st>>>((const Ti*)in, (To*)out, D, N, out2, D2,
                                                                           in_scale, sidx);
                else
                    stage_mix_q_kernel<Ti, To, QQ, false><<<gq, b, 0, st>>>((const Ti*)in, (To*)out, D, N, out2,
                                                                            D2, in_scale, sidx);
            };
            if (dtype_in == RK_FP64 && dtype_out == RK_FP64) go(double{}, double{});
            else if (dtype_in == RK_FP64) go(double{}, float{});
            else if (dtype_out == RK_FP64) go(float{}, double{});
            else go(float{}, float{});
            return hipGetLastError();
        });
        return e;
    }
    if (dtype_in == RK_FP64 && dtype_out == RK_FP64)
        stage_mix_kernel<double, double><<<g, b, 0, st>>>((const double*)in, (double*)out, D, qout, qin, N, out2, D2, in_scale, sidx);
    else if (dtype_in == RK_FP64 && dtype_out == RK_FP32)
        stage_mix_kernel<double, float><<<g, b, 0, st>>>((const double*)in, (float*)out, D, qout, qin, N, out2, D2, in_scale, sidx);
    else if (dtype_in == RK_FP32 && dtype_out == RK_FP64)
        stage_mix_kernel<float, double><<<g, b, 0, st>>>((const float*)in, (double*)out, D, qout, qin, N, out2, D2, in_scale, sidx);
    else
        stage_mix_kernel<float, float><<<g, b, 0, st>>>((const float*)in, (float*)out, D, qout, qin, N, out2, D2, in_scale, sidx);
    return hipGetLastError();
}

hipError_t launch_rhs_mix(const double* G, const double* w, double* out, const double* c1,
                          const double* c2, int Q, int N, hipStream_t st) {
    const long long n3 = (long long)N * N * N;
    rhs_mix_kernel<<<grid_for(n3), kBlock, 0, st>>>(G, w, out, c1, c2, Q, N);
    return hipGetLastError();
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// V2 paths need 16-byte aligned vector bases and an even leading dimension;
// segments at odd offsets are handled element-wise at their ends.
hipError_t launch_dots(const double* X, int nvec, long long ld, const double* w, const Segs& sg, int self,
                       double* part, int nblocks, hipStream_t st) {
    const int nout = nvec + self;
    const bool v2 = aligned16(w) && (nvec == 0 || (aligned16(X) && ld % 2 == 0));
    if (nvec == 0) {
        if (v2) dots_kernel<0, true><<<nblocks, kBlock, 0, st>>>(X, ld, w, sg, self, part, nout, 0);
        else dots_kernel<0, false><<<nblocks, kBlock, 0, st>>>(X, ld, w, sg, self, part, nout, 0);
        return hipGetLastError();
    }
    for (int l0 = 0; l0 < nvec; l0 += kChunk) {
        const int nv = std::min(kChunk, nvec - l0);
        const int sf = (self && l0 + nv == nvec) ? 1 : 0;
        const double* Xc = X + (long long)l0 * ld;
        hipError_t e = dispatch_nv(nv, [&](auto NV) {
            if (v2) dots_kernel<NV, true><<<nblocks, kBlock, 0, st>>>(Xc, ld, w, sg, sf, part, nout, l0);
            else dots_kernel<NV, false><<<nblocks, kBlock, 0, st>>>(Xc, ld, w, sg, sf, part, nout, l0);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_gs_update(const double* X, int nvec, long long ld, const double* h, int hstride,
                            const double* sig, const double* w, double* out, const Segs& sg, double* norm_part,
                            int nblocks, hipStream_t st) {
    const bool v2 = aligned16(X) && aligned16(w) && aligned16(out) && ld % 2 == 0;
    if (nvec <= 0) return hipErrorInvalidValue;
    for (int l0 = 0; l0 < nvec; l0 += kChunk) {
        const int nv = std::min(kChunk, nvec - l0);
        const bool last = l0 + nv == nvec;
        const double* Xc = X + (long long)l0 * ld;
        const double* src = l0 == 0 ? w : out;
        const double* sc = sig ? sig + (long long)l0 * kSigStride : nullptr;
        double* np = last ? norm_part : nullptr;
        hipError_t e = dispatch_nv(nv, [&](auto NV) {
            if (v2)
                gs_update_kernel<NV, true><<<nblocks, kBlock, 0, st>>>(Xc, ld, h + l0, hstride, sc, src, out, sg, np);
            else
                gs_update_kernel<NV, false><<<nblocks, kBlock, 0, st>>>(Xc, ld, h + l0, hstride, sc, src, out, sg, np);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reduce(const double* part, int nblocks, int nout, double* out, int accumulate,
                         hipStream_t st, const double* scale, int nscale, double* inv_sqrt_out, int ngroup,
                         int ostride) {
    reduce_kernel<<<dim3(nout, ngroup), kBlock, 0, st>>>(part, nblocks, nout, out, ostride, accumulate, scale,
                                                         nscale, inv_sqrt_out);
    return hipGetLastError();
}

hipError_t launch_combine(double* kv, int dtype_z, const void* Z, int nz, long long ld, const double* y,
                          int ystride, const Segs& sg, hipStream_t st) {
    const size_t es = dtype_z == RK_FP64 ? 8 : 4;
    const bool v2 = aligned16(kv) && (reinterpret_cast<uintptr_t>(Z) % (2 * es)) == 0 && ld % 2 == 0;
    long long n = 0;
    for (int q = 0; q < sg.first[sg.ngroup]; ++q) n += sg.len[q];
    const int nb = grid_for(n / 2 + 1);
    for (int l0 = 0; l0 < nz; l0 += kChunk) {
        const int nv = std::min(kChunk, nz - l0);
        const char* Zc = static_cast<const char*>(Z) + (size_t)l0 * ld * es;
        hipError_t e = dispatch_nv(nv, [&](auto NV) {
            if (dtype_z == RK_FP64) {
                const double* z = reinterpret_cast<const double*>(Zc);
                if (v2) combine_kernel<NV, double, true><<<nb, kBlock, 0, st>>>(kv, z, ld, y + l0, ystride, sg);
                else combine_kernel<NV, double, false><<<nb, kBlock, 0, st>>>(kv, z, ld, y + l0, ystride, sg);
            } else {
                const float* z = reinterpret_cast<const float*>(Zc);
                if (v2) combine_kernel<NV, float, true><<<nb, kBlock, 0, st>>>(kv, z, ld, y + l0, ystride, sg);
                else combine_kernel<NV, float, false><<<nb, kBlock, 0, st>>>(kv, z, ld, y + l0, ystride, sg);
            }
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_stage_combine(double* y, const double* kv, const double* b, double tau, int Q,
                                int N, hipStream_t st) {
    BVec bv;
    for (int i = 0; i < RK_MAX_Q; ++i) bv.v[i] = i < Q ? b[i] : 0.0;
    const long long n3 = (long long)N * N * N;
    stage_combine_kernel<<<grid_for(n3), kBlock, 0, st>>>(y, kv, bv, tau, Q, N);
    return hipGetLastError();
}

hipError_t launch_fill(int dtype, void* x, long long n, double value, hipStream_t st) {
    if (dtype == RK_FP64) fill_kernel<double><<<grid_for(n), kBlock, 0, st>>>((double*)x, n, value);
    else fill_kernel<float><<<grid_for(n), kBlock, 0, st>>>((float*)x, n, (float)value);
    return hipGetLastError();
}

hipError_t launch_sub_from(double* v, const double* b, long long n, hipStream_t st) {
    sub_from_kernel<<<grid_for(n), kBlock, 0, st>>>(v, b, n);
    return hipGetLastError();
}

hipError_t launch_copy(int dtype, const void* src, void* dst, long long n, hipStream_t st) {
    if (dtype == RK_FP64) copy_kernel<double><<<grid_for(n), kBlock, 0, st>>>((const double*)src, (double*)dst, n);
    else copy_kernel<float><<<grid_for(n), kBlock, 0, st>>>((const float*)src, (float*)dst, n);
    return hipGetLastError();
}

hipError_t launch_power_partial(int k, int dtype, const StageScal& sc, const void* v, const void* w, void* z,
                                int n, int nstage, double* part, int nblocks, hipStream_t st, const void* dMv,
                                const void* dKv) {
    if (dtype == RK_FP64)
        power_partial_kernel<double><<<nblocks, kBlock, 0, st>>>(to_scal<double>(sc), k, (const double*)v, (const double*)w, (double*)z, n, nstage, part, (const double*)dMv, (const double*)dKv);
    else
        power_partial_kernel<float><<<nblocks, kBlock, 0, st>>>(to_scal<float>(sc), k, (const float*)v, (const float*)w, (float*)z, n, nstage, part, (const float*)dMv, (const float*)dKv);
    return hipGetLastError();
}

hipError_t launch_power_normalize(int dtype, const void* z, void* v, const double* red, int N, int nstage,
                                  hipStream_t st) {
    const long long N3 = (long long)N * N * N;
    if (dtype == RK_FP64)
        power_normalize_kernel<double><<<grid_for(N3 * nstage), kBlock, 0, st>>>((const double*)z, (double*)v, red, N3, nstage);
    else
        power_normalize_kernel<float><<<grid_for(N3 * nstage), kBlock, 0, st>>>((const float*)z, (float*)v, red, N3, nstage);
    return hipGetLastError();
}

hipError_t launch_random_fill(int dtype, void* x, int N, int nstage, unsigned seed, hipStream_t st) {
    const long long N3 = (long long)N * N * N;
    if (dtype == RK_FP64)
        random_fill_kernel<double><<<grid_for(N3 * nstage), kBlock, 0, st>>>((double*)x, N, nstage, seed);
    else
        random_fill_kernel<float><<<grid_for(N3 * nstage), kBlock, 0, st>>>((float*)x, N, nstage, seed);
    return hipGetLastError();
}

}  // namespace rk
