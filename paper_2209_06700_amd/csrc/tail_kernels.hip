// The coarse end of the multigrid V-cycle in one launch (Sec. 5.4: one
// V-cycle per stage block, all blocks batched).
//
// Below a size threshold every level of the V-cycle is a chain of small
// launches whose cost is their own latency, not their work: per level the
// smoothing steps, the residual, the two transfers and the coarse solve are
// each a launch over a few thousand nodes.  tail_vcycle_kernel runs the whole
// V-cycle from such a level down to the coarsest one and back up in one
// launch, one workgroup per stage block.  The workgroup walks the same steps
// as the multi-launch path (Chebyshev-Jacobi pre-smoothing from zero, residual,
// restriction, the coarser levels, prolongation and add, post-smoothing; the
// coarsest level a Chebyshev-Jacobi solve from zero), with the same buffer
// rotation, so the result lands where the caller expects it.
//
// Every operator application is sum factorisation over the whole level in
// three passes through a per-block scratch of four arrays (the 1D banded
// global matrices along x, then y, then z, with the epilogue fused into the z
// pass), each pass ended by a workgroup barrier; the transfers are three 1D
// passes each.  The scratch lives in LDS for levels of up to 17^3 nodes,
// else in memory.  The level vectors stay in the context's level buffers
// ([Q][N^3], x fastest); the data of these levels are a few hundred kilobytes
// and stay in the caches.
//
// Dirichlet conditions: inputs are read as zero on boundary nodes, and every
// vector the kernel writes gets zeros on its boundary nodes.

#include <hip/hip_runtime.h>

#include "op_kernel.h"
#include "rk_internal.h"
#include "transfer_rows.h"

namespace rk {
namespace dev {
namespace {

constexpr int kTailThreads = 1024;

// Chebyshev update at one node (the multi-launch path's formula):
//   x_new = x + ca (x - xo) + cb D^-1 (b - A x)
template <typename T>
__device__ __forceinline__ T cheb_node(T b, T x, T xo, T ax, T rD, T ca, T cb) {
    return x + ca * (x - xo) + cb * (b - ax) * rD;
}

// The steps of one stage block's V-cycle on the tail levels: s is the block,
// X1, X2, S, Tz the four scratch arrays (n3max values each, n3max at least the
// node count of the largest tail level).
template <int K, typename T>
struct Tail {
    int s;
    T* X1;
    T* X2;
    T* S;
    T* Tz;

    __device__ Tail(int stage, T* scratch, long long n3max)
        : s(stage), X1(scratch), X2(scratch + n3max), S(scratch + 2 * n3max), Tz(scratch + 3 * n3max) {}

    static __device__ __forceinline__ T dm(int i) { return diag_rt<K, 0, T>(i % K); }
    static __device__ __forceinline__ T dk(int i) { return diag_rt<K, 1, T>(i % K); }

    // Jacobi diagonal of alpha M + beta K at interior node (x, y, z).
    static __device__ __forceinline__ T diag(T alpha, T beta, int x, int y, int z) {
        const T mx = dm(x), my = dm(y), mz = dm(z);
        return alpha * mx * my * mz + beta * (dk(x) * my * mz + mx * dk(y) * mz + mx * my * dk(z));
    }

    // v = epi(alpha Mref u + beta Kref u) on level lv, for this block.
    // EPI_RESID: v = b - A u.  EPI_CHEB: v = cheb_node(b, u, xo, A u, 1/D)
    // (xo null: zero).  Ends with a barrier.
    template <int EPI>
    __device__ __forceinline__ void apply(const TailLevel& L, const T* u, T* v, const T* b, const T* xo, T ca, T cb) {
        const int n = L.n, N = n * K + 1, nK = N - 1;
        const int NN = N * N;
        const T alpha = T(L.alpha[s]), beta = T(L.beta[s]);
        const int tid = threadIdx.x;
        const int M = N - 2;                     // interior nodes per direction
        // x pass: rows (z, y) interior, element e along x
        for (int it = tid; it < M * M * n; it += kTailThreads) {
            const int e = it % n, r = it / n;
            const int y = r % M + 1, z = r / M + 1;
            const T* row = u + (long long)z * NN + (long long)y * N;
            T w[2 * K + 1], mx[K], kx[K];
#pragma unroll
            for (int j = 0; j <= 2 * K; ++j) {
                const int x = (e - 1) * K + j;
                w[j] = (x > 0 && x < nK) ? row[x] : T(0);
            }
            row_apply<K, 0, T>(w, mx);
            row_apply<K, 1, T>(w, kx);
            T* o1 = X1 + (long long)z * NN + (long long)y * N;
            T* o2 = X2 + (long long)z * NN + (long long)y * N;
#pragma unroll
            for (int c = 0; c < K; ++c) {
                o1[e * K + c] = fma(alpha, mx[c], beta * kx[c]);
                o2[e * K + c] = beta * mx[c];
            }
        }
        __syncthreads();
        // y pass: (z interior, element e along y, x interior)
        for (int it = tid; it < M * n * M; it += kTailThreads) {
            const int x = it % M + 1, r = it / M;
            const int e = r % n, z = r / n + 1;
            const long long zo = (long long)z * NN + x;
            T w1[2 * K + 1], w2[2 * K + 1], m1[K], k2[K], t2[K];
#pragma unroll
            for (int j = 0; j <= 2 * K; ++j) {
                const int y = (e - 1) * K + j;
                const bool ok = y > 0 && y < nK;
                w1[j] = ok ? X1[zo + (long long)y * N] : T(0);
                w2[j] = ok ? X2[zo + (long long)y * N] : T(0);
            }
            row_apply<K, 0, T>(w1, m1);
            row_apply<K, 1, T>(w2, k2);
            row_apply<K, 0, T>(w2, t2);
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const long long o = zo + (long long)(e * K + c) * N;
                S[o] = m1[c] + k2[c];
                Tz[o] = t2[c];
            }
        }
        __syncthreads();
        // z pass and epilogue: (element e along z, every column (y, x)); the
        // boundary nodes of v are written as zero, the top plane by e = n - 1
        for (int it = tid; it < n * NN; it += kTailThreads) {
            const int col = it % NN, e = it / NN;
            const int y = col / N, x = col - y * N;
            const bool inner = x > 0 && x < nK && y > 0 && y < nK;
            T ms[K], kt[K];
            if (inner) {
                T ws[2 * K + 1], wt[2 * K + 1];
#pragma unroll
                for (int j = 0; j <= 2 * K; ++j) {
                    const int z = (e - 1) * K + j;
                    const bool ok = z > 0 && z < nK;
                    ws[j] = ok ? S[(long long)z * NN + col] : T(0);
                    wt[j] = ok ? Tz[(long long)z * NN + col] : T(0);
                }
                row_apply<K, 0, T>(ws, ms);
                row_apply<K, 1, T>(wt, kt);
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int z = e * K + c;
                const long long g = (long long)z * NN + col;
                T out = T(0);
                if (inner && z > 0) {
                    const T av = ms[c] + kt[c];
                    if (EPI == EPI_RESID) {
                        out = b[g] - av;
                    } else {
                        const T rD = T(1) / diag(alpha, beta, x, y, z);
                        out = cheb_node(b[g], u[g], xo ? xo[g] : T(0), av, rD, ca, cb);
                    }
                }
                v[g] = out;
            }
            if (e == n - 1) v[(long long)nK * NN + col] = T(0);
        }
        __syncthreads();
    }

    // v = c0 D^-1 b (the first Chebyshev iterate from zero).  Ends with a barrier.
    __device__ __forceinline__ void first_iterate(const TailLevel& L, const T* b, T* v, T c0) {
        const int N = L.n * K + 1, nK = N - 1;
        const T alpha = T(L.alpha[s]), beta = T(L.beta[s]);
        const long long N3 = (long long)N * N * N;
        for (long long g = threadIdx.x; g < N3; g += kTailThreads) {
            const int x = (int)(g % N), r = (int)(g / N);
            const int y = r % N, z = r / N;
            const bool inner = x > 0 && x < nK && y > 0 && y < nK && z > 0 && z < nK;
            v[g] = inner ? c0 * b[g] / diag(alpha, beta, x, y, z) : T(0);
        }
        __syncthreads();
    }

    // Chebyshev-Jacobi smoothing of degree L.degree on level L (Saad,
    // Alg. 12.1, the multi-launch path's recurrence): from zero (x_1 =
    // c0 D^-1 b in `first`) or from the iterate in `first`.  x_j lands in
    // `first` for odd j and in `second` for even j from zero, the other way
    // round otherwise.  Returns the buffer of the last iterate.
    __device__ __forceinline__ T* chebyshev(const TailLevel& L, const T* b, T* first, T* second, bool zero_start) {
        const double theta = L.theta, delta = L.delta, sigma = L.sigma;
        const T c0 = T(1.0 / theta);
        T* cur;
        T* prev;
        bool prev_zero;
        if (zero_start) {
            first_iterate(L, b, first, c0);
            cur = first; prev = second; prev_zero = true;     // x_0 = 0
        } else {
            apply<EPI_CHEB>(L, first, second, b, nullptr, T(0), c0);
            cur = second; prev = first; prev_zero = false;
        }
        double rho = 1.0 / sigma;
        for (int j = 1; j < L.degree; ++j) {
            const double rho_new = 1.0 / (2.0 * sigma - rho);
            const T ca = T(rho_new * rho), cb = T(2.0 * rho_new / delta);
            // x_{j+1} overwrites x_{j-1} (each node reads its own old value first)
            apply<EPI_CHEB>(L, cur, prev, b, prev_zero ? nullptr : prev, ca, cb);
            T* t = prev; prev = cur; cur = t;
            prev_zero = false;
            rho = rho_new;
        }
        return cur;
    }

    // b_c = P^T r from level F (fine) to level C: three 1D passes through X1, X2.
    __device__ __forceinline__ void restrict_to(const TailLevel& F, const TailLevel& C, const T* r, T* bc) {
        const int nc = C.n, Nc = nc * K + 1, Nf = 2 * nc * K + 1;
        const int tid = threadIdx.x;
        const int Mf = Nf - 2, Mc = Nc - 2;
        // x: fine rows (zf, yf) interior -> X1[zf][yf][xc], xc < Nc - 1
        for (int it = tid; it < Mf * Mf * nc; it += kTailThreads) {
            const int E = it % nc, rr = it / nc;
            const int yf = rr % Mf + 1, zf = rr / Mf + 1;
            const T* row = r + ((long long)zf * Nf + yf) * Nf;
            T w[4 * K + 1], o[K];
#pragma unroll
            for (int t = 0; t <= 4 * K; ++t) {
                const int xf = 2 * (E - 1) * K + t;
                w[t] = (xf > 0 && xf < Nf - 1) ? row[xf] : T(0);
            }
            xfer::rrow<K, T>(w, o);
            T* dst = X1 + ((long long)zf * Nf + yf) * Nc;
#pragma unroll
            for (int c = 0; c < K; ++c) dst[E * K + c] = o[c];
        }
        __syncthreads();
        // y: (zf interior, E, xc interior) -> X2[zf][yc][xc], yc < Nc - 1
        for (int it = tid; it < Mf * nc * Mc; it += kTailThreads) {
            const int xc = it % Mc + 1, rr = it / Mc;
            const int E = rr % nc, zf = rr / nc + 1;
            T w[4 * K + 1], o[K];
#pragma unroll
            for (int t = 0; t <= 4 * K; ++t) {
                const int yf = 2 * (E - 1) * K + t;
                w[t] = (yf > 0 && yf < Nf - 1) ? X1[((long long)zf * Nf + yf) * Nc + xc] : T(0);
            }
            xfer::rrow<K, T>(w, o);
#pragma unroll
            for (int c = 0; c < K; ++c) X2[((long long)zf * Nc + E * K + c) * Nc + xc] = o[c];
        }
        __syncthreads();
        // z: (E, every coarse column) -> bc, boundary nodes zero
        const int NNc = Nc * Nc;
        for (int it = tid; it < nc * NNc; it += kTailThreads) {
            const int col = it % NNc, E = it / NNc;
            const int yc = col / Nc, xc = col - yc * Nc;
            const bool inner = xc > 0 && xc < Nc - 1 && yc > 0 && yc < Nc - 1;
            T o[K];
            if (inner) {
                T w[4 * K + 1];
#pragma unroll
                for (int t = 0; t <= 4 * K; ++t) {
                    const int zf = 2 * (E - 1) * K + t;
                    w[t] = (zf > 0 && zf < Nf - 1) ? X2[((long long)zf * Nc + yc) * Nc + xc] : T(0);
                }
                xfer::rrow<K, T>(w, o);
            }
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const int zc = E * K + c;
                bc[(long long)zc * NNc + col] = (inner && zc > 0) ? o[c] : T(0);
            }
            if (E == nc - 1) bc[(long long)(Nc - 1) * NNc + col] = T(0);
        }
        __syncthreads();
    }

    // x_f += P x_c from level C to level F: three 1D passes through X1, X2.
    __device__ __forceinline__ void prolong_add(const TailLevel& C, const T* xc, T* xf) {
        const int nc = C.n, Nc = nc * K + 1, Nf = 2 * nc * K + 1;
        const int tid = threadIdx.x;
        const int Mc = Nc - 2, Mf = Nf - 2;
        constexpr int J2 = 2 * K;
        // x: coarse rows (zc, yc) interior -> X1[zc][yc][xf], 0 < xf < Nf - 1
        for (int it = tid; it < Mc * Mc * nc; it += kTailThreads) {
            const int E = it % nc, rr = it / nc;
            const int yc = rr % Mc + 1, zc = rr / Mc + 1;
            const T* row = xc + ((long long)zc * Nc + yc) * Nc;
            T w[K + 1];
#pragma unroll
            for (int a = 0; a <= K; ++a) {
                const int x = E * K + a;
                w[a] = (x > 0 && x < Nc - 1) ? row[x] : T(0);
            }
            T* dst = X1 + ((long long)zc * Nc + yc) * Nf;
            xfer::tfor<J2>([&](auto jm) {
                constexpr int j = decltype(jm)::value;
                T v = T(xfer::PE<K, j, 0>::v) * w[0];
                xfer::tfor<K>([&](auto am) {
                    constexpr int a = decltype(am)::value + 1;
                    v = fma(T(xfer::PE<K, j, a>::v), w[a], v);
                });
                dst[E * J2 + j] = v;
            });
        }
        __syncthreads();
        // y: (zc interior, E, xf interior) -> X2[zc][yf][xf]
        for (int it = tid; it < Mc * nc * Mf; it += kTailThreads) {
            const int x = it % Mf + 1, rr = it / Mf;
            const int E = rr % nc, zc = rr / nc + 1;
            T w[K + 1];
#pragma unroll
            for (int a = 0; a <= K; ++a) {
                const int y = E * K + a;
                w[a] = (y > 0 && y < Nc - 1) ? X1[((long long)zc * Nc + y) * Nf + x] : T(0);
            }
            xfer::tfor<J2>([&](auto jm) {
                constexpr int j = decltype(jm)::value;
                T v = T(xfer::PE<K, j, 0>::v) * w[0];
                xfer::tfor<K>([&](auto am) {
                    constexpr int a = decltype(am)::value + 1;
                    v = fma(T(xfer::PE<K, j, a>::v), w[a], v);
                });
                X2[((long long)zc * Nf + E * J2 + j) * Nf + x] = v;
            });
        }
        __syncthreads();
        // z: (E, fine column interior) -> xf += ..., interior fine nodes only
        const int NNf = Nf * Nf;
        for (int it = tid; it < nc * Mf * Mf; it += kTailThreads) {
            const int x = it % Mf + 1, rr = it / Mf;
            const int y = rr % Mf + 1, E = rr / Mf;
            T w[K + 1];
#pragma unroll
            for (int a = 0; a <= K; ++a) {
                const int z = E * K + a;
                w[a] = (z > 0 && z < Nc - 1) ? X2[((long long)z * Nf + y) * Nf + x] : T(0);
            }
            xfer::tfor<J2>([&](auto jm) {
                constexpr int j = decltype(jm)::value;
                const int zf = E * J2 + j;
                if (zf > 0) {
                    T v = T(xfer::PE<K, j, 0>::v) * w[0];
                    xfer::tfor<K>([&](auto am) {
                        constexpr int a = decltype(am)::value + 1;
                        v = fma(T(xfer::PE<K, j, a>::v), w[a], v);
                    });
                    const long long g = (long long)zf * NNf + (long long)y * Nf + x;
                    xf[g] += v;
                }
            });
        }
        __syncthreads();
    }
};

// Levels of up to kTailLdsNodes nodes keep the four scratch arrays in LDS
// (4 * 17^3 values: 79 KB in fp32, 157 KB in fp64, within gfx950's 160 KB per
// workgroup); larger first levels use the per-block scratch in memory.
constexpr int kTailLdsNodes = 17 * 17 * 17;

template <int K, typename T, bool LDS>
__global__ void __launch_bounds__(kTailThreads) tail_vcycle_kernel(TailArgs a) {
    const int s = a.s0 + blockIdx.x;
    T* scratch;
    if constexpr (LDS) {
        __shared__ T lds[4 * kTailLdsNodes];
        scratch = lds;
    } else {
        scratch = static_cast<T*>(a.scratch) + (long long)s * a.sstride;
    }
    Tail<K, T> t(s, scratch, a.n3max);
    auto at = [&](void* base, const TailLevel& L) { return static_cast<T*>(base) + (long long)s * L.N3; };
    // down: pre-smoothing (result in `first`), residual into `second`, restriction
    for (int l = 0; l + 1 < a.nlev; ++l) {
        const TailLevel& L = a.lv[l];
        T* b = at(L.b, L);
        T* first = at(L.x, L);
        T* second = at(L.y, L);
        T* pre = t.chebyshev(L, b, first, second, true);
        T* spare = pre == first ? second : first;
        t.template apply<EPI_RESID>(L, pre, spare, b, nullptr, T(0), T(0));
        t.restrict_to(L, a.lv[l + 1], spare, at(a.lv[l + 1].b, a.lv[l + 1]));
    }
    // coarsest level: Chebyshev-Jacobi from zero
    const TailLevel& Lc = a.lv[a.nlev - 1];
    T* res = t.chebyshev(Lc, at(Lc.b, Lc), at(Lc.x, Lc), at(Lc.y, Lc), true);
    // up: prolongation + add into the pre-smoothed iterate, post-smoothing
    for (int l = a.nlev - 2; l >= 0; --l) {
        const TailLevel& L = a.lv[l];
        T* b = at(L.b, L);
        T* first = at(L.x, L);
        T* second = at(L.y, L);
        // the pre-smoothed iterate: x_nu lands in `first` for odd nu
        T* pre = (L.degree % 2 == 1) ? first : second;
        T* spare = pre == first ? second : first;
        t.prolong_add(a.lv[l + 1], res, pre);
        res = t.chebyshev(L, b, pre, spare, false);
    }
}

template <int K>
hipError_t launch_tail_k(const TailArgs& a, int nblocks, hipStream_t st) {
    const bool lds = a.n3max <= kTailLdsNodes;
    if (a.dtype == RK_FP64) {
        if (lds) tail_vcycle_kernel<K, double, true><<<nblocks, kTailThreads, 0, st>>>(a);
        else tail_vcycle_kernel<K, double, false><<<nblocks, kTailThreads, 0, st>>>(a);
    } else {
        if (lds) tail_vcycle_kernel<K, float, true><<<nblocks, kTailThreads, 0, st>>>(a);
        else tail_vcycle_kernel<K, float, false><<<nblocks, kTailThreads, 0, st>>>(a);
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace dev

hipError_t launch_tail_vcycle(int k, const TailArgs& a, int nblocks, hipStream_t st) {
    if (a.nlev < 1 || a.nlev > kTailMaxLevels || nblocks < 1) return hipErrorInvalidValue;
    switch (k) {
        case 1: return dev::launch_tail_k<1>(a, nblocks, st);
        case 2: return dev::launch_tail_k<2>(a, nblocks, st);
        case 3: return dev::launch_tail_k<3>(a, nblocks, st);
        case 4: return dev::launch_tail_k<4>(a, nblocks, st);
        case 5: return dev::launch_tail_k<5>(a, nblocks, st);
        case 6: return dev::launch_tail_k<6>(a, nblocks, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk
