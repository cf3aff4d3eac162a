// Matrix-free application of the stage operators on the uniform Q_k mesh.
//
// On the uniform hexahedral mesh the assembled mass and stiffness matrices are
// sums of Kronecker products of 1D matrices (the element integrals separate
// and every cell is a translate of the reference cube):
//     M = m (x) m (x) m,   K = a (x) m (x) m + m (x) a (x) m + m (x) m (x) a,
// where m and a are the 1D global mass and stiffness matrices, which are
// assembled from the (k+1) x (k+1) element matrices Mhat, Khat.  The kernel
// therefore evaluates the operator by sum factorisation over the whole grid:
// one banded 1D product per direction and term, with no element gather/scatter
// and no write conflicts (every output node is owned by exactly one thread).
//
// Operator for output stage s (per-stage scales in the kernel arguments, 1D
// element matrices as compile-time constants, cell size folded into scales):
//   diagonal mix:  v_s = alpha_s Mref u_s  + beta_s Kref u_s
//   pair mix:      v_s = alpha_s Mref uM_s + beta_s Kref uK_s
// with Mref = Mhat (x) Mhat (x) Mhat and Kref the matching stiffness sum.  The
// pair form takes two input vectors; the Q x Q stage mixes of the dense
// operators (A^-1 (x) M, A (x) K) are applied to the inputs by a streaming
// kernel beforehand, so this kernel never reads more than two inputs per node.
//
// Sum factorisation (per node plane), wM / wK the mass / stiffness inputs:
//   X1 = alpha Mhat_x wM + beta Khat_x wK,  X2 = beta Mhat_x wK   (x-pass)
//   S  = Mhat_y X1 + Khat_y X2,             T  = Mhat_y X2          (y-pass)
//   v  = Mhat_z S + Khat_z T                                       (z)
//
// Work decomposition (one workgroup):
//   * an x-y tile of TX x TY output nodes (element aligned; about 32 or 64
//     nodes wide, 8 elements tall, 4 for k >= 5) and a z-chunk of cz
//     elements, both chosen per level by the autotuner; all Q stages of one
//     tile are consecutive workgroups on one XCD (shared halo reads in that
//     XCD's L2);
//   * the workgroup marches up the z-chunk one node plane at a time:
//       1. the input plane tile plus a halo of k nodes below and 1 above in x
//          and y is staged in LDS (zero outside the interior: Dirichlet); the
//          loads of a plane are issued ahead, into registers;
//       2. x-pass: every (row, x-element) item applies the 1D matrices to the
//          2k+1 inputs it needs and writes k outputs to LDS;
//       3. y-pass: every thread owns one x column and a y-pencil of k nodes
//          (one element; for k >= 5 two threads share a pencil, each with
//          half of its rows) and applies the 1D matrices along y from LDS;
//       4. z: the plane's results are accumulated element by element into k+1
//          per-thread registers per pencil node; when an element's top plane
//          has been added, k output planes are complete and are written (with
//          the epilogue: store, residual or Chebyshev update).
//   With double-buffered LDS (fp32) one iteration does the y-pass of plane
//   q-1, the x-pass of plane q and the staging of plane q+1 behind a single
//   barrier; fp64 keeps single buffers (half the LDS, more resident
//   workgroups) and two barriers.  The z-chunk re-reads the k planes of the
//   element below it.
// One work item is op_tile; op_kernel runs one item per workgroup for one
// problem, op_list_kernel walks the items of several problems of one degree
// (different meshes, Q and scales) on a persistent grid.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>

#include "element_data.h"
#include "rk_internal.h"

namespace rk {
namespace dev {

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1.
template <typename F, int... I>
__device__ __forceinline__ void cfor_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void cfor(F&& f) {
    cfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Entry (A, B) of the 1D element mass (W = 0) or stiffness (W = 1) matrix.
template <int K, int W, int A, int B>
struct EC {
    static constexpr double v = W == 0 ? elem::Table<K>::d.M[A][B] : elem::Table<K>::d.A[A][B];
};

// Diagonal of the 1D global matrix at a node with local index R (R = 0 is an
// interior vertex shared by two cells).
template <int K, int W, int R>
struct DG {
    static constexpr double v = R == 0 ? EC<K, W, 0, 0>::v + EC<K, W, K, K>::v : EC<K, W, R, R>::v;
};

// Tile shapes (TS): 0 = about 32 x-nodes, 1 = about 64 x-nodes (fp32
// diagonal-mix kernels only), both 8 pencils tall (4 for k >= 5, whose
// pencils are split).  The autotuner picks one per level and epilogue class.
template <int K, int TS = 0>
struct Tile {
    static constexpr int CX = ((TS == 1 ? 64 : 32) / K) > 0 ? ((TS == 1 ? 64 : 32) / K) : 1;  // elements in x
    static constexpr int TX = CX * K;                       // owned nodes in x
    // pencils per tile in y (taller tiles cut the x-pass halo rows but leave
    // fewer resident workgroups per CU, which measured slower).  Split
    // pencils (k >= 5, below) take two threads each: 4 pencils keep a
    // workgroup at 4 waves (8 with the 64-wide tile), so that the three
    // waves per SIMD that the fp64 kernels' registers allow hold three
    // workgroups per CU instead of one of 8 waves.
    static constexpr int CY = K >= 5 ? 4 : 8;
    static constexpr int TY = CY * K;                       // owned nodes in y
    // Pencil split: for k >= 5 the K rows of a y-pencil are shared by two
    // threads (rows 0..R-1 and R..K-1), which halves the per-thread
    // accumulators and y-pass outputs; each half is a whole number of waves,
    // so the two halves never share a wave.
    static constexpr int SPL = K >= 5 ? 2 : 1;
    static constexpr int R = (K + SPL - 1) / SPL;           // pencil rows per thread
    static constexpr int NTH = SPL == 1 ? TX * CY : (TX * CY + 63) / 64 * 64;   // threads per half
    static constexpr int NT = SPL * NTH;                    // threads
    static constexpr int RW = TX + K + 1;                   // staged input width
    // LDS pitches are 2 (mod 4): lanes of a 16-lane group then read
    // adjacent pairs (ds_read2) from distinct banks
    static constexpr int RX = RW + ((2 - RW % 4) + 4) % 4;  // staged row pitch
    static constexpr int RY = TY + K + 1;                   // staged input height
    static constexpr int XP = RY + ((2 - RY % 4) + 4) % 4;  // X1/X2 column pitch (stored x-major)
};

template <typename T>
struct OpArgs {
    const T* u;       // input (both terms for the diagonal mix; mass term for the pair)
    const T* u2;      // pair mix: stiffness-term input
    T* v;
    const T* b;
    const T* xo;
    long long stride;
    int n, s0, nstage;
    int tiles_x, tiles_y, chunks_z, nwork, per_xcd;
    int cz;                                       // elements per z-chunk
    int xo_zero, xo_from_b;
    T ca, cb, icb, c0;                            // Chebyshev coefficients, icb = 1/cb
    T alpha[RK_MAX_Q], beta[RK_MAX_Q];            // per-stage scales
};

// out[a] = (E w)[a] for the k nodes eK..eK+k-1 of element e, where
// w[0..2k] holds the inputs at nodes (e-1)k .. (e+1)k.  The vertex eK
// collects row k of element e-1 and row 0 of element e.
template <int K, int W, typename T>
__device__ __forceinline__ void row_apply(const T* w, T* out) {
    T o = T(EC<K, W, K, 0>::v) * w[0];
    cfor<K - 1>([&](auto bm) {
        constexpr int b = decltype(bm)::value + 1;
        o = fma(T(EC<K, W, K, b>::v), w[b], o);
    });
    o = fma(T(EC<K, W, K, K>::v + EC<K, W, 0, 0>::v), w[K], o);
    cfor<K>([&](auto bm) {
        constexpr int b = decltype(bm)::value + 1;
        o = fma(T(EC<K, W, 0, b>::v), w[K + b], o);
    });
    out[0] = o;
    cfor<K - 1>([&](auto am) {
        constexpr int a = decltype(am)::value + 1;
        T q = T(EC<K, W, a, 0>::v) * w[K];
        cfor<K>([&](auto bm) {
            constexpr int b = decltype(bm)::value + 1;
            q = fma(T(EC<K, W, a, b>::v), w[K + b], q);
        });
        out[a] = q;
    });
}

// out[i] = (E w)[A0 + i], i < RR, for rows A0 + i < K of the element (row 0
// the shared vertex, as in row_apply; rows >= 1 read only w[K..2K]); rows
// past K are 0.
template <int K, int W, int A0, int RR, typename T>
__device__ __forceinline__ void row_apply_rows(const T* w, T* out) {
    cfor<RR>([&](auto im) {
        constexpr int a = A0 + decltype(im)::value;
        if constexpr (a == 0) {
            T o = T(EC<K, W, K, 0>::v) * w[0];
            cfor<K - 1>([&](auto bm) {
                constexpr int b = decltype(bm)::value + 1;
                o = fma(T(EC<K, W, K, b>::v), w[b], o);
            });
            o = fma(T(EC<K, W, K, K>::v + EC<K, W, 0, 0>::v), w[K], o);
            cfor<K>([&](auto bm) {
                constexpr int b = decltype(bm)::value + 1;
                o = fma(T(EC<K, W, 0, b>::v), w[K + b], o);
            });
            out[decltype(im)::value] = o;
        } else if constexpr (a < K) {
            T q = T(EC<K, W, a, 0>::v) * w[K];
            cfor<K>([&](auto bm) {
                constexpr int b = decltype(bm)::value + 1;
                q = fma(T(EC<K, W, a, b>::v), w[K + b], q);
            });
            out[decltype(im)::value] = q;
        } else {
            out[decltype(im)::value] = T(0);
        }
    });
}

// 1D diagonals at a runtime local index r in [0, K)
template <int K, int W, typename T>
__device__ __forceinline__ T diag_rt(int r) {
    T d = T(DG<K, W, 0>::v);
    cfor<K - 1>([&](auto rm) {
        constexpr int rr = decltype(rm)::value + 1;
        if (r == rr) d = T(DG<K, W, rr>::v);
    });
    return d;
}

// Minimum waves per SIMD requested from the register allocator: four for the
// fp32 Chebyshev kernels of degree <= 4, which hold the epilogue prefetch on
// top of the operator's registers (measured 13% faster than the three waves
// the allocator picks by itself, at the cost of a few loop-invariant values
// spilled outside the march).  Otherwise the allocator's own choice.
template <int K, typename T, int EPI>
struct MinWaves {
    static constexpr int v = (sizeof(T) == 4 && K <= 4 && (EPI == EPI_CHEB || EPI == EPI_CHEB1)) ? 4 : 1;
};

// One work item w < p.nwork of the operator: the x-y tile, z-chunk and
// stage that w encodes (stage fastest, then tile x, tile y, chunk).
template <int K, typename T, int MIX, int EPI, int TS>
__device__ __forceinline__ void op_tile(const OpArgs<T>& p, const int w) {
    using TL = Tile<K, TS>;
    constexpr int P = K + 1;
    constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT, RX = TL::RX, RY = TL::RY;
    constexpr int XP = TL::XP, CX = TL::CX;
    constexpr int SPL = TL::SPL, R = TL::R, NTH = TL::NTH;
    constexpr int NU = MIX == MIX_PAIR ? 2 : 1;
    constexpr bool CHEB = EPI == EPI_CHEB || EPI == EPI_CHEB1;
    constexpr bool INB = EPI == EPI_CHEB1;               // input x1 = c0 D^-1 b, formed from b
    constexpr int NBUF = sizeof(T) == 4 ? 2 : 1;          // LDS buffers per array
    constexpr int NSLOT = (RY * RX + NT - 1) / NT;      // staged values per thread
    constexpr int NXIT = (RY * CX + NT - 1) / NT;       // x-pass items per thread
    constexpr int USZ = NU * RY * RX, XSZ = TX * XP;
    __shared__ T sU[NBUF * USZ];
    __shared__ T sX1[NBUF * XSZ];
    __shared__ T sX2[NBUF * XSZ];

    int rem = w;
    const int sl = rem % p.nstage;
    rem /= p.nstage;
    const int itx = rem % p.tiles_x;
    rem /= p.tiles_x;
    const int ity = rem % p.tiles_y;
    const int icz = rem / p.tiles_y;
    const int s = p.s0 + sl;

    const int n = p.n, nK = n * K, N = nK + 1;
    const long long NN = (long long)N * N;
    const int CZ = p.cz;
    const int TZ = CZ * K;
    const int X0 = itx * TX, Y0 = ity * TY, E0 = icz * CZ, Z0 = E0 * K;
    const int tid = threadIdx.x;
    // pencil half h (uniform per wave) and this thread's x column and rows
    // a0 .. a0 + nr - 1 of y-pencil py; threads past the tile's TX CY columns
    // (the padding of a half to whole waves) own no column
    const int h = SPL == 1 ? 0 : tid / NTH;
    const int tl = tid - h * NTH;
    const bool has_col = SPL == 1 || tl < TX * TL::CY;
    const int tx = tl % TX, py = tl / TX;
    const int a0 = h * R, nr = K - a0 < R ? K - a0 : R;
    const int gx = X0 + tx, gy0 = Y0 + py * K + a0;
    // vs may alias p.xo (in-place Chebyshev update), so it is not restrict.
    T* vs = p.v + (long long)s * p.stride;
    // 32-bit in-plane offset of this thread's first pencil node, and the same
    // in bytes (N^2 sizeof(T) < 2^32): accesses are a uniform 64-bit plane or
    // row base plus a 32-bit per-lane byte offset
    const unsigned colbase = (unsigned)gy0 * (unsigned)N + (unsigned)gx;
    const unsigned colbyte = colbase * (unsigned)sizeof(T);

    // Tiles that own only far-boundary nodes: write the zeros and leave.
    if (X0 >= nK || Y0 >= nK || Z0 >= nK) {
        const int z1 = min(Z0 + TZ, N);
        if (has_col && gx < N)
            for (int z = Z0; z < z1; ++z) {
                T* pl = vs + z * NN;
#pragma unroll
                for (int a = 0; a < R; ++a)
                    if (a < nr && gy0 + a < N) pl[colbase + (unsigned)(a * N)] = T(0);
            }
        return;
    }

    const T alpha = p.alpha[s];
    const T beta = p.beta[s];
    const T* __restrict__ us = p.u + (long long)s * p.stride;
    const T* __restrict__ us2 = MIX == MIX_PAIR ? p.u2 + (long long)s * p.stride : nullptr;

    // 1 / D for the Chebyshev steps (fp32: hardware reciprocal; the
    // smoother is a preconditioner, so the last-bit rounding is immaterial)
    auto recip = [](T d) __attribute__((always_inline)) {
        if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(d);
        else return T(1) / d;
    };

    // Load slots of this thread: in-plane byte offset and validity (interior in x, y).
    unsigned soff[NSLOT];
    unsigned smask = 0;
#pragma unroll
    for (int m = 0; m < NSLOT; ++m) {
        const int i = tid + m * NT;
        const int r = i / RX, c = i - r * RX;
        const int xx = X0 - K + c, yy = Y0 - K + r;
        const bool ok = i < RY * RX && c < TL::RW && xx > 0 && xx < nK && yy > 0 && yy < nK;
        soff[m] = ok ? ((unsigned)yy * (unsigned)N + (unsigned)xx) * (unsigned)sizeof(T) : 0u;
        smask |= ok ? (1u << m) : 0u;
    }
    T pre[NU][NSLOT];
    // Fused first Chebyshev step: the staged input is x1 = c0 D^-1 b.  Per
    // slot D = pa dMz + pb dKz with pa, pb from the slot's x and y position
    // and dMz, dKz (1D diagonals at the plane's z) held for the issued plane.
    T pa[INB ? NSLOT : 1], pb[INB ? NSLOT : 1];
    T izm = T(1), izk = T(0);
    if constexpr (INB) {
#pragma unroll
        for (int m = 0; m < NSLOT; ++m) {
            const int i = tid + m * NT;
            const int r = i / RX, c = i - r * RX;
            const int rx = (X0 + c) % K, ry = (Y0 + r) % K;   // (X0 - K + c) mod K, X0 a multiple of K
            const T mx = diag_rt<K, 0, T>(rx), kx = diag_rt<K, 1, T>(rx);
            const T my = diag_rt<K, 0, T>(ry), ky = diag_rt<K, 1, T>(ry);
            const bool ok = smask >> m & 1u;
            pa[m] = ok ? fma(alpha, mx * my, beta * fma(kx, my, mx * ky)) : T(1);
            pb[m] = ok ? beta * mx * my : T(0);
        }
    }
    // Issue the loads of plane z into registers.  Every slot loads from a
    // valid address (offset 0 for slots outside the interior); the zeros of
    // those slots are selected when the plane is committed to LDS, one
    // iteration later, so that no instruction here waits for the loads.
    auto issue = [&](int z) __attribute__((always_inline)) {
        if constexpr (INB) {
            izm = diag_rt<K, 0, T>(z % K);
            izk = diag_rt<K, 1, T>(z % K);
        }
        if (z > 0 && z < nK) {
            const char* __restrict__ pl = reinterpret_cast<const char*>(us + z * NN);
#pragma unroll
            for (int m = 0; m < NSLOT; ++m) pre[0][m] = *reinterpret_cast<const T*>(pl + soff[m]);
            if (MIX == MIX_PAIR) {
                const char* __restrict__ pl2 = reinterpret_cast<const char*>(us2 + z * NN);
#pragma unroll
                for (int m = 0; m < NSLOT; ++m) pre[NU - 1][m] = *reinterpret_cast<const T*>(pl2 + soff[m]);
            }
        } else {
#pragma unroll
            for (int m = 0; m < NSLOT; ++m)
#pragma unroll
                for (int j = 0; j < NU; ++j) pre[j][m] = T(0);
        }
    };
    auto commit = [&](int buf) __attribute__((always_inline)) {
        T* dst = sU + buf * USZ;
#pragma unroll
        for (int m = 0; m < NSLOT; ++m) {
            const int i = tid + m * NT;
            if (m < NSLOT - 1 || i < RY * RX) {
                const bool ok = smask >> m & 1u;
                if constexpr (INB) dst[i] = ok ? pre[0][m] * (p.c0 * recip(fma(pa[m], izm, pb[m] * izk))) : T(0);
                else dst[i] = ok ? pre[0][m] : T(0);
                if (MIX == MIX_PAIR) dst[RY * RX + i] = ok ? pre[NU - 1][m] : T(0);
            }
        }
    };

    T acc[P][R];
    T sv[R], tv[R];

    // x-pass of the plane staged in sU[buf] -> sX1/sX2[buf]
    auto xpass = [&](int buf) __attribute__((always_inline)) {
        const T* U = sU + buf * USZ;
        T* X1 = sX1 + buf * XSZ;
        T* X2 = sX2 + buf * XSZ;
#pragma unroll
        for (int q = 0; q < NXIT; ++q) {
            const int it = tid + q * NT;
            if (q < NXIT - 1 || it < RY * CX) {
                const int cx = it / RY, r = it - cx * RY;
                T wv[2 * K + 1], mx[K], kx[K];
                const T* src = &U[r * RX + cx * K];
#pragma unroll
                for (int j = 0; j <= 2 * K; ++j) wv[j] = src[j];
                T* o1 = &X1[cx * K * XP + r];
                T* o2 = &X2[cx * K * XP + r];
                if (MIX == MIX_DIAG) {
                    row_apply<K, 0, T>(wv, mx);
                    row_apply<K, 1, T>(wv, kx);
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        o1[a * XP] = fma(alpha, mx[a], beta * kx[a]);
                        o2[a * XP] = beta * mx[a];
                    }
                } else {
                    T wk[2 * K + 1], mk[K];
                    const T* src2 = src + RY * RX;
#pragma unroll
                    for (int j = 0; j <= 2 * K; ++j) wk[j] = src2[j];
                    row_apply<K, 0, T>(wv, mx);
                    row_apply<K, 1, T>(wk, kx);
                    row_apply<K, 0, T>(wk, mk);
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        o1[a * XP] = fma(alpha, mx[a], beta * kx[a]);
                        o2[a * XP] = beta * mk[a];
                    }
                }
            }
        }
    };
    // y-pass of sX1/sX2[buf] for this thread's pencil rows -> sv, tv
    // (rows A0 .. A0 + R - 1; rows >= 1 read only the element's own K + 1
    // inputs)
    auto ypass_rows = [&](const T* X1, const T* X2, int cb, auto a0m) __attribute__((always_inline)) {
        constexpr int A0 = decltype(a0m)::value;
        constexpr int J0 = A0 == 0 ? 0 : K;
        T w1[2 * K + 1], w2[2 * K + 1], m1[R], k2[R];
#pragma unroll
        for (int j = 0; j <= 2 * K; ++j) {
            w1[j] = j >= J0 ? X1[cb + j] : T(0);
            w2[j] = j >= J0 ? X2[cb + j] : T(0);
        }
        row_apply_rows<K, 0, A0, R, T>(w1, m1);
        row_apply_rows<K, 1, A0, R, T>(w2, k2);
        row_apply_rows<K, 0, A0, R, T>(w2, tv);
#pragma unroll
        for (int a = 0; a < R; ++a) sv[a] = m1[a] + k2[a];
    };
    auto ypass = [&](int buf) __attribute__((always_inline)) {
        const T* X1 = sX1 + buf * XSZ;
        const T* X2 = sX2 + buf * XSZ;
        if constexpr (SPL == 1) {
            T w1[2 * K + 1], w2[2 * K + 1], m1[K], k2[K];
#pragma unroll
            for (int j = 0; j <= 2 * K; ++j) {
                w1[j] = X1[tx * XP + py * K + j];
                w2[j] = X2[tx * XP + py * K + j];
            }
            row_apply<K, 0, T>(w1, m1);
            row_apply<K, 1, T>(w2, k2);
            row_apply<K, 0, T>(w2, tv);
#pragma unroll
            for (int a = 0; a < K; ++a) sv[a] = m1[a] + k2[a];
        } else {
            if (!has_col) return;
            const int cb = tx * XP + py * K;
            if (h == 0) ypass_rows(X1, X2, cb, std::integral_constant<int, 0>{});
            else ypass_rows(X1, X2, cb, std::integral_constant<int, R>{});
        }
    };

    // acc[c][a] += Mhat[c][B] sv[a] + Khat[c][B] tv[a]  (B compile-time)
    auto zacc = [&](auto bm) __attribute__((always_inline)) {
        constexpr int B = decltype(bm)::value;
        cfor<P>([&](auto cm) {
            constexpr int c = decltype(cm)::value;
#pragma unroll
            for (int a = 0; a < R; ++a)
                acc[c][a] = fma(T(EC<K, 0, c, B>::v), sv[a], fma(T(EC<K, 1, c, B>::v), tv[a], acc[c][a]));
        });
    };
    // acc[c][a] = Mhat[c][0] sv[a] + Khat[c][0] tv[a]
    auto zinit = [&]() __attribute__((always_inline)) {
        cfor<P>([&](auto cm) {
            constexpr int c = decltype(cm)::value;
#pragma unroll
            for (int a = 0; a < R; ++a)
                acc[c][a] = fma(T(EC<K, 0, c, 0>::v), sv[a], T(EC<K, 1, c, 0>::v) * tv[a]);
        });
    };

    // Epilogue data.  Boundary status of the thread's nodes in x and y.
    const bool colok = has_col && gx < N;
    const bool xbnd = gx == 0 || gx == nK;
    T dmx = T(0), dkx = T(0);
    if (CHEB) {
        const int rx = gx % K;
        dmx = diag_rt<K, 0, T>(rx);
        dkx = diag_rt<K, 1, T>(rx);
    }
    const T* __restrict__ bs = (EPI != EPI_STORE) ? p.b + (long long)s * p.stride : nullptr;
    const T* xos = (CHEB && !p.xo_zero && !p.xo_from_b) ? p.xo + (long long)s * p.stride : nullptr;

    // Jacobi diagonal of the block operator at node (c, a) of the pencil:
    //   D = alpha dMx dMy dMz + beta (dKx dMy dMz + dMx dKy dMz + dMx dMy dKz)
    //     = C1 (alpha dMx + beta dKx) + C2 beta dMx,
    // C1 = dMy dMz and C2 = dKy dMz + dMy dKz compile-time constants; the
    // per-thread factors may carry a common scale.
    auto jac_s = [&](auto cm, auto am, T u1, T u2) __attribute__((always_inline)) {
        constexpr int c = decltype(cm)::value;
        constexpr int a = decltype(am)::value;
        constexpr T C1 = T(DG<K, 0, a>::v * DG<K, 0, c>::v);
        constexpr T C2 = T(DG<K, 1, a>::v * DG<K, 0, c>::v + DG<K, 0, a>::v * DG<K, 1, c>::v);
        return fma(C1, u1, C2 * u2);
    };
    const T ju1 = fma(alpha, dmx, beta * dkx), ju2 = beta * dmx;
    auto jac = [&](auto cm, auto am) __attribute__((always_inline)) { return jac_s(cm, am, ju1, ju2); };

    const int E1 = min(E0 + CZ, n);                    // chunk elements E0 .. E1-1
    // Pencils whose nodes are all interior in x and y take the branch-free path.
    const bool pencil_inner = colok && !xbnd && gy0 > 0 && gy0 + nr - 1 < nK;
    // Chebyshev update x + ca (x - x_prev) + cb D^-1 (b - A x) at one node
    // (rD = 1/D); x = c0 D^-1 b for the fused first step, x_prev = c0 D^-1 b
    // when the previous iterate is the first one.
    auto cheb_update = [&](T b, T x, T xo, T av, T rD) __attribute__((always_inline)) {
        if (INB) x = p.c0 * b * rD;
        if (!INB && p.xo_from_b) xo = p.c0 * b * rD;
        return x + p.ca * (x - xo) + p.cb * (b - av) * rD;
    };
    // Entry of a vector at this thread's column in the row that starts at
    // element offset ro (uniform 64-bit row base + 32-bit lane byte offset).
    auto at = [&](const T* base, long long ro) __attribute__((always_inline)) -> const T& {
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + ro) + colbyte);
    };
    // Epilogue prefetch (fp32 march, residual and Chebyshev epilogues): the
    // epilogue inputs of output plane c of an element are fetched in the
    // iteration that x-passes that plane and, in the next one, subtracted
    // from the accumulator of that output (acc = A x - epre), so the writes
    // wait on no load.  x itself comes from the staged plane in LDS (no second
    // read from memory).  For the Chebyshev update
    //   out = x + ca (x - x_prev) + cb D^-1 (b - A x) = (cb / D) (epre - A x),
    //   epre = b + (x + ca (x - x_prev)) D / cb;
    // for the residual epre = b.
    constexpr bool PF = EPI != EPI_STORE && NBUF == 2 && K <= 4;   // registers allow it up to Q_4
    T fb[K], fx[K], fo[K];
#pragma unroll
    for (int a = 0; a < K; ++a) { fb[a] = T(0); fx[a] = T(0); fo[a] = T(0); }

    // x_prev = c0 D^-1 b:  epre = b (1 - ca c0 / cb) + (1 + ca) x D / cb
    const T opc = T(1) + p.ca, k1 = T(1) - p.ca * p.c0 * p.icb;
    // fused first step (x = c0 D^-1 b, x_prev = 0):  epre = b (1 + (1 + ca) c0 / cb)
    const T kb1 = T(1) + opc * p.c0 * p.icb;
    // fetch the epilogue inputs of output plane c of element ee, whose input
    // plane is staged in sU[buf] (fast-path lanes of flushed elements only)
    auto pf_issue = [&](int ee, int c, int buf) __attribute__((always_inline)) {
        if (colok && ee >= E0 && ee < E1) {
            const long long zo = (long long)(ee * K + c) * NN;
            const T* U = sU + buf * USZ + (py * K + K) * RX + tx + K;
            cfor<K>([&](auto am) {
                constexpr int a = decltype(am)::value;
                const long long ro = zo + (long long)a * N;
                const bool rv = gy0 + a < N;              // rows past the grid: nothing to load
                fb[a] = rv ? at(bs, ro) : T(0);
                if (CHEB && !INB) {            // the fused first step needs b only
                    fx[a] = U[a * RX];
                    fo[a] = (rv && xos) ? at(xos, ro) : T(0);
                }
            });
        }
    };
    // fold the inputs fetched for output plane c into its accumulators
    auto pf_fold = [&](auto cm) __attribute__((always_inline)) {
        constexpr int c = decltype(cm)::value;
        if constexpr (PF) {
            cfor<K>([&](auto am) {
                constexpr int a = decltype(am)::value;
                T e;
                if (EPI == EPI_RESID) e = fb[a];
                else if (INB) e = fb[a] * kb1;  // x = c0 D^-1 b, x_prev = 0
                else if (p.xo_from_b)   // x_prev = c0 D^-1 b
                    e = fma(fx[a] * opc, (jac_s(cm, am, ju1, ju2) * p.icb), fb[a] * k1);
                else e = fma(fma(p.ca, fx[a] - fo[a], fx[a]), (jac_s(cm, am, ju1, ju2) * p.icb), fb[a]);
                acc[c][a] -= e;
            });
        }
    };

    // Write this thread's rows A0 .. A0 + R - 1 (those < K) of the K
    // completed output planes of element e.  Per output plane the epilogue
    // loads of its rows are issued together before any use.
    auto flush_rows = [&](int e, auto a0m) __attribute__((always_inline)) {
        constexpr int A0 = decltype(a0m)::value;
        if (pencil_inner && e > 0) {
            cfor<K>([&](auto cm) {
                constexpr int c = decltype(cm)::value;
                const long long zo = (long long)(e * K + c) * NN;
                T lb[R], lx[R], lo[R];
                if (EPI != EPI_STORE) {
                    cfor<R>([&](auto am) {
                        constexpr int a = decltype(am)::value;
                        if constexpr (A0 + a < K) {
                            const long long ro = zo + (long long)a * N;
                            lb[a] = at(bs, ro);
                            if (CHEB) {
                                lx[a] = INB ? T(0) : at(us, ro);
                                lo[a] = xos ? at(xos, ro) : T(0);
                            }
                        }
                    });
                }
                cfor<R>([&](auto am) {
                    constexpr int a = decltype(am)::value;
                    if constexpr (A0 + a < K) {
                        const long long ro = zo + (long long)a * N;     // uniform row offset
                        const T av = acc[c][a];
                        T out;
                        if (EPI == EPI_STORE) out = av;
                        else if (EPI == EPI_RESID) out = lb[a] - av;
                        else out = cheb_update(lb[a], lx[a], lo[a], av,
                                               recip(jac(cm, std::integral_constant<int, A0 + a>{})));
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(vs + ro) + colbyte) = out;
                    }
                });
            });
            return;
        }
        if (!colok) return;
        cfor<K>([&](auto cm) {
            constexpr int c = decltype(cm)::value;
            const int z = e * K + c;
            const long long zo = (long long)z * NN;
            cfor<R>([&](auto am) {
                constexpr int a = decltype(am)::value;
                if constexpr (A0 + a < K) {
                    const int y = gy0 + a;
                    if (y < N) {
                        const unsigned off = colbase + (unsigned)(a * N);
                        const bool bnd = z == 0 || xbnd || y == 0 || y == nK;
                        T out = T(0);
                        if (!bnd) {
                            const T av = acc[c][a];
                            const long long g = zo + off;
                            if (EPI == EPI_STORE) out = av;
                            else if (EPI == EPI_RESID) out = bs[g] - av;
                            else {
                                const T x = INB ? T(0) : us[g];
                                const T xo = xos ? xos[g] : T(0);
                                out = cheb_update(bs[g], x, xo, av,
                                                  recip(jac(cm, std::integral_constant<int, A0 + a>{})));
                            }
                        }
                        (vs + zo)[off] = out;
                    }
                }
            });
        });
    };

    // Write the K completed output planes of element e.  Per output plane the
    // epilogue loads of its K nodes are issued together before any use.
    auto flush = [&](int e) __attribute__((always_inline)) {
        if constexpr (PF) {
            // every column of the tile (boundary nodes written as zero)
            if (!colok) return;
            cfor<K>([&](auto cm) {
                constexpr int c = decltype(cm)::value;
                const int z = e * K + c;
                const long long zo = (long long)z * NN;
                cfor<K>([&](auto am) {
                    constexpr int a = decltype(am)::value;
                    const int y = gy0 + a;
                    if (y < N) {
                        const long long ro = zo + (long long)a * N;
                        const bool bnd = z == 0 || xbnd || y == 0 || y >= nK;
                        const T d = -acc[c][a];                      // epre - A x
                        const T out = EPI == EPI_RESID ? d : p.cb * recip(jac(cm, am)) * d;
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(vs + ro) + colbyte) = bnd ? T(0) : out;
                    }
                });
            });
            return;
        }
        if constexpr (SPL == 1) {
            flush_rows(e, std::integral_constant<int, 0>{});
        } else {
            if (h == 0) flush_rows(e, std::integral_constant<int, 0>{});
            else flush_rows(e, std::integral_constant<int, R>{});
        }
    };

    // z-accumulation of the plane just y-passed.  B is the plane's index
    // within the current element e (compile time: the march is unrolled by
    // element, so no accumulator is selected at run time); B = 0 starts the
    // first element of the chunk.  When the element's top plane (B = K) has
    // been added, its K output planes are written and the top plane's
    // contribution carries over as the bottom plane of element e+1.
    int e = 0;
    auto zplane = [&](auto bm) __attribute__((always_inline)) {
        constexpr int B = decltype(bm)::value;
        if constexpr (B == 0) {
            zinit();
        } else {
            // this plane is output plane B of element e (B < K) or plane 0 of e+1
            if constexpr (PF && B < K) pf_fold(bm);
            zacc(bm);
            if constexpr (B == K) {
                if (e >= E0) flush(e);
                T carry[R];
#pragma unroll
                for (int a = 0; a < R; ++a) carry[a] = acc[K][a];
                zinit();
#pragma unroll
                for (int a = 0; a < R; ++a) acc[0][a] += carry[a];
                ++e;
                if constexpr (PF) pf_fold(std::integral_constant<int, 0>{});
            }
        }
    };
    // after zplane(B) (plane eK+B, or eK with e advanced when B = K): fetch
    // the epilogue inputs of the next plane, staged in sU[buf]
    auto pf_next = [&](auto bm, int buf) __attribute__((always_inline)) {
        constexpr int B = decltype(bm)::value;
        constexpr int CN = (B == K || B == 0) ? 1 : B + 1;
        if constexpr (PF) {
            if constexpr (CN == K) pf_issue(e + 1, 0, buf);
            else pf_issue(e, CN, buf);
        }
    };

    // March up the chunk over the planes zbeg .. zend (NP = NE K + 1 planes,
    // NE >= 1 elements), each processed once.  Plane p >= 1 has index
    // B = (p - 1) mod K + 1 within its element; the last plane has B = K.
    const int ebeg = E0 > 0 ? E0 - 1 : 0;
    const int NE = E1 - ebeg;
    const int zbeg = ebeg * K;
    const int NP = NE * K + 1;
    e = ebeg;
    using I0 = std::integral_constant<int, 0>;
    using IK = std::integral_constant<int, K>;
    if constexpr (NBUF == 2) {
        // Iteration q: y-pass + z-accumulation of plane q-1, x-pass of plane
        // q, staging of plane q+1 (loaded during iteration q-1), loads of
        // plane q+2; then one barrier.  The phases use disjoint buffers.
        auto iter = [&](int q, auto bm) __attribute__((always_inline)) {
            // q is kept opaque (an empty asm in a scalar register): otherwise
            // the buffer parity folds to a constant in each unrolled copy and
            // every copy keeps its own LDS addresses live (more VGPRs).
            asm volatile("" : "+s"(q));
            ypass((q - 1) & 1);
            zplane(bm);
            pf_next(bm, q & 1);
            xpass(q & 1);
            if (q + 1 < NP) {
                commit((q + 1) & 1);
                if (q + 2 < NP) issue(zbeg + q + 2);
            }
            __syncthreads();
        };
        issue(zbeg);
        commit(0);
        issue(zbeg + 1);
        __syncthreads();
        xpass(0);
        commit(1);
        if (NP > 2) issue(zbeg + 2);
        __syncthreads();
        iter(1, I0{});
        for (int g = 0; g < NE; ++g) {
            cfor<K>([&](auto bm) {
                constexpr int B = decltype(bm)::value + 1;
                const int q = 2 + g * K + (B - 1);
                if (q < NP) iter(q, std::integral_constant<int, B>{});
            });
        }
        ypass((NP - 1) & 1);
        zplane(IK{});
    } else {
        // Iteration q: stage plane q (loaded during iteration q-1), loads of
        // plane q+1, y-pass + z-accumulation of plane q-1; barrier; x-pass of
        // plane q; barrier.  (fp64 keeps a run-time plane index: the unrolled
        // march needs more registers here and costs occupancy.)
        int b = 0;
        auto zstep = [&](bool first) __attribute__((always_inline)) {
            if (first) {
                zinit();
            } else {
                cfor<K>([&](auto bm) {
                    constexpr int B = decltype(bm)::value + 1;
                    if (b == B) zacc(std::integral_constant<int, B>{});
                });
            }
            if (b == K) {
                if (e >= E0) flush(e);
                T carry[R];
#pragma unroll
                for (int a = 0; a < R; ++a) carry[a] = acc[K][a];
                zinit();
#pragma unroll
                for (int a = 0; a < R; ++a) acc[0][a] += carry[a];
                ++e;
                b = 0;
            }
            ++b;
        };
        issue(zbeg);
        for (int q = 0; q < NP; ++q) {
            commit(0);
            if (q + 1 < NP) issue(zbeg + q + 1);
            if (q > 0) {
                ypass(0);
                zstep(q == 1);
            }
            __syncthreads();
            xpass(0);
            __syncthreads();
        }
        ypass(0);
        zstep(false);
    }
    // The chunk that contains the top boundary plane writes it.
    if (E0 + CZ > n && colok) {
        T* pl = vs + (long long)nK * NN;
#pragma unroll
        for (int a = 0; a < R; ++a)
            if (a < nr && gy0 + a < N) pl[colbase + (unsigned)(a * N)] = T(0);
    }
}

// One workgroup per work item; consecutive items (the Q stages of a tile)
// go to one XCD (the hardware deals workgroups to the 8 XCDs round robin).
template <int K, typename T, int MIX, int EPI, int TS>
__global__ void __launch_bounds__((Tile<K, TS>::NT), (MinWaves<K, T, EPI>::v)) op_kernel(OpArgs<T> p) {
    const int bid = blockIdx.x;
    const int w = (bid & 7) * p.per_xcd + (bid >> 3);
    if (w >= p.nwork) return;
    op_tile<K, T, MIX, EPI, TS>(p, w);
}

// Work list over several problems of one degree: the items of problem i are
// start[i] .. start[i+1]-1 of the list.  The kernel is persistent: a fixed
// grid (a multiple of 8 workgroups) walks the list, workgroup b taking the
// items of its XCD's contiguous range (b mod 8) in steps of grid/8, so the
// stages and neighbouring tiles of a problem meet in one L2 as in op_kernel.
template <typename T>
struct OpListArgs {
    int count, total, per_xcd;
    int start[kOpListMax + 1];
    OpArgs<T> e[kOpListMax];
};

template <int K, typename T>
__global__ void __launch_bounds__((Tile<K, 0>::NT)) op_list_kernel(OpListArgs<T> a) {
    const int b = blockIdx.x, step = gridDim.x >> 3;
    for (int j = b >> 3; j < a.per_xcd; j += step) {
        const int w = (b & 7) * a.per_xcd + j;
        if (w >= a.total) break;                       // the rest of this range is past the list
        int i = 0;
        while (i + 1 < a.count && a.start[i + 1] <= w) ++i;
        op_tile<K, T, MIX_DIAG, EPI_STORE, 0>(a.e[i], w - a.start[i]);
        __syncthreads();                               // LDS is reused by the next item
    }
}

// Fills the launch fields of p (tiles, z-chunk, work count) for tile shape TS.
template <int K, typename T, int TS>
void op_setup(const OpLaunch& L, OpArgs<T>& p) {
    using TL = Tile<K, TS>;
    p.u = static_cast<const T*>(L.u);
    p.u2 = static_cast<const T*>(L.u2);
    p.v = static_cast<T*>(L.v);
    p.b = static_cast<const T*>(L.b);
    p.xo = static_cast<const T*>(L.xo);
    p.stride = L.stride;
    p.n = L.n;
    p.s0 = L.s0;
    p.nstage = L.nstage;
    const int N = L.n * K + 1;
    p.tiles_x = (N + TL::TX - 1) / TL::TX;
    p.tiles_y = (N + TL::TY - 1) / TL::TY;
    // z-chunk length: long enough to amortise the k re-read planes, short
    // enough to give every CU several workgroups
    int cz = 16;
    while (cz > 1 && (long long)p.tiles_x * p.tiles_y * ((L.n + cz - 1) / cz) * L.nstage < 2048) cz /= 2;
    if (L.cz > 0) cz = L.cz;                                                           // tuned or set
    p.cz = cz;
    p.chunks_z = (N + cz * K - 1) / (cz * K);
    p.nwork = p.tiles_x * p.tiles_y * p.chunks_z * L.nstage;
    p.per_xcd = (p.nwork + 7) / 8;
    p.xo_zero = L.xo == nullptr;
    p.ca = T(L.ca);
    p.cb = T(L.cb);
    p.icb = L.cb != 0.0 ? T(1.0 / L.cb) : T(0);
    p.c0 = T(L.c0);
    p.xo_from_b = L.xo_from_b;
    for (int i = 0; i < RK_MAX_Q; ++i) {
        p.alpha[i] = T(L.alpha[i]);
        p.beta[i] = T(L.beta[i]);
    }
}

template <int K, typename T>
hipError_t launch_op_list_typed(const OpLaunch* L, int count, hipStream_t st) {
    OpListArgs<T> a{};
    a.count = count;
    a.start[0] = 0;
    for (int i = 0; i < count; ++i) {
        op_setup<K, T, 0>(L[i], a.e[i]);
        a.start[i + 1] = a.start[i] + a.e[i].nwork;
    }
    a.total = a.start[count];
    a.per_xcd = (a.total + 7) / 8;
    // persistent grid: at most kOpListGrid workgroups, a multiple of 8
    const int grid = 8 * std::min(a.per_xcd, kOpListGrid / 8);
    op_list_kernel<K, T><<<grid, Tile<K, 0>::NT, 0, st>>>(a);
    return hipGetLastError();
}

// The diagonal-mix store form for the problems L[0..count) of degree K, all
// of one dtype, in one launch (count <= kOpListMax).
template <int K>
hipError_t launch_op_list_k(const OpLaunch* L, int count, hipStream_t st) {
    if (count < 1 || count > kOpListMax) return hipErrorInvalidValue;
    for (int i = 0; i < count; ++i)
        if (L[i].k != K || L[i].dtype != L[0].dtype || L[i].mix != MIX_DIAG || L[i].epi != EPI_STORE)
            return hipErrorInvalidValue;
    return L[0].dtype == RK_FP64 ? launch_op_list_typed<K, double>(L, count, st)
                                 : launch_op_list_typed<K, float>(L, count, st);
}

template <int K, typename T, int TS>
hipError_t launch_op_shape(const OpLaunch& L) {
    using TL = Tile<K, TS>;
    OpArgs<T> p;
    op_setup<K, T, TS>(L, p);
    dim3 grid(8 * p.per_xcd), block(TL::NT);
#define RK_OP_CASE(MX, EP)                                                      \
    if (L.mix == MX && L.epi == EP) {                                           \
        op_kernel<K, T, MX, EP, TS><<<grid, block, 0, L.stream>>>(p);           \
        return hipGetLastError();                                               \
    }
    RK_OP_CASE(MIX_DIAG, EPI_STORE)
    RK_OP_CASE(MIX_DIAG, EPI_RESID)
    RK_OP_CASE(MIX_DIAG, EPI_CHEB)
    RK_OP_CASE(MIX_DIAG, EPI_CHEB1)
    if constexpr (TS == 0) {
        RK_OP_CASE(MIX_PAIR, EPI_STORE)
        RK_OP_CASE(MIX_PAIR, EPI_RESID)
    }
#undef RK_OP_CASE
    return hipErrorInvalidValue;
}

template <int K, typename T>
hipError_t launch_op_typed(const OpLaunch& L) {
    if constexpr (sizeof(T) == 4) {
        if (L.ts == 1 && L.mix == MIX_DIAG) return launch_op_shape<K, T, 1>(L);
    }
    if (L.ts != 0 && L.ts != 1) return hipErrorInvalidValue;
    return launch_op_shape<K, T, 0>(L);
}

template <int K>
hipError_t launch_op_k(const OpLaunch& L) {
    return L.dtype == RK_FP64 ? launch_op_typed<K, double>(L) : launch_op_typed<K, float>(L);
}

}  // namespace dev
}  // namespace rk
