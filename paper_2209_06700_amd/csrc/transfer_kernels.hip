// Fused multigrid transfers between the n-cell and 2n-cell grids of degree k.
//
// The prolongation is the embedding of the nested Q_k spaces, which on the
// uniform grid is a tensor product P = P1 (x) P1 (x) P1 of the 1D
// interpolation P1: within coarse cell E the fine nodes 2Ek + j (j = 0..2k)
// take  sum_a Pe[j][a] x_c[Ek + a]  (Pe[j][a] = l_a at the fine node).
//
// prolong_add_kernel: x_fine += P x_coarse in one pass.  A workgroup owns a
// fine x-y tile (whole coarse cells) and a chunk of coarse cells in z.  It
// marches over the coarse planes of its chunk; each plane is staged in LDS,
// interpolated in x (LDS) and in y (registers), so that each thread holds the
// x-y interpolants of the k+1 coarse planes of the current coarse cell for its
// fine nodes; the 2k fine planes of the cell are then formed in registers
// and added to the fine vector (one read and one write per fine node).
//
// Restriction x_coarse = P^T x_fine in two passes: restrict_xy_kernel
// restricts every fine plane in x and y (one workgroup per plane tile, fine
// plane plus the fine halo of one coarse cell staged in LDS), writing an
// intermediate of coarse x-y size per fine plane; restrict_z_kernel then
// restricts along z.  In 1D, coarse node Ek + a collects
//   sum_{t=0}^{2k} Pe[t][a] f(2Ek + t)              (a = 1..k-1), and the vertex
//   a = 0 also  sum_{t=0}^{2k-1} Pe[t][k] f(2(E-1)k + t),
// each fine node counted once (the fine vertex 2Ek has Pe[0][0] = 1).  Coarse
// boundary nodes are written as zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "element_data.h"
#include "rk_internal.h"
#include "transfer_rows.h"

namespace rk {
namespace {

using xfer::PE;
using xfer::rrow;
using xfer::tfor;

template <int K>
struct PTile {
    static constexpr int CC = (16 / K) > 0 ? (16 / K) : 1;   // coarse cells per tile side
    static constexpr int TF = 2 * K * CC;                      // fine nodes per tile side
    static constexpr int RC = CC * K + 1;                      // coarse nodes staged per side
    static constexpr int TPY = 8;                              // thread rows
    static constexpr int NT = TF * TPY;                        // threads
    static constexpr int RPT = (TF + TPY - 1) / TPY;           // fine rows per thread
    static constexpr int XP = TF + 1;                          // padded LDS row
};

template <typename T>
struct ProlongArgs {
    const T* coarse;
    T* fine;
    long long cstride, fstride;   // stage strides
    int nc;                       // coarse cells per direction
    int tiles, chunks, czc, nwork, per_xcd;
};

template <int K, typename T>
__global__ void __launch_bounds__(PTile<K>::NT) prolong_add_kernel(ProlongArgs<T> p) {
    using TL = PTile<K>;
    constexpr int TF = TL::TF, RC = TL::RC, NT = TL::NT, RPT = TL::RPT, XP = TL::XP;
    constexpr int P1 = K + 1, J2 = 2 * K;
    __shared__ T sC[RC * RC];
    __shared__ T sXL[RC * XP];
    __shared__ T sP[(2 * K + 1) * P1];

    const int bid = blockIdx.x;
    const int w = (bid & 7) * p.per_xcd + (bid >> 3);
    if (w >= p.nwork) return;
    int rem = w;
    const int itx = rem % p.tiles;
    rem /= p.tiles;
    const int ity = rem % p.tiles;
    rem /= p.tiles;
    const int icz = rem % p.chunks;
    const int s = rem / p.chunks;

    const int nc = p.nc, Nc = nc * K + 1, Nf = 2 * nc * K + 1;
    const long long NNc = (long long)Nc * Nc, NNf = (long long)Nf * Nf;
    const T* __restrict__ cs = p.coarse + (long long)s * p.cstride;
    T* fs = p.fine + (long long)s * p.fstride;
    const int tid = threadIdx.x;
    const int tx = tid % TF, ty = tid / TF;
    const int X0c = itx * (RC - 1), Y0c = ity * (RC - 1);
    const int X0f = itx * TF, Y0f = ity * TF;
    const int E0 = icz * p.czc, E1 = min(E0 + p.czc, nc);

    for (int i = tid; i < (2 * K + 1) * P1; i += NT) {
        const int j = i / P1, a = i - j * P1;
        T v = T(0);
        tfor<2 * K + 1>([&](auto jm) {
            tfor<P1>([&](auto am) {
                if (j == decltype(jm)::value && a == decltype(am)::value)
                    v = T(PE<K, decltype(jm)::value, decltype(am)::value>::v);
            });
        });
        sP[i] = v;
    }

    // x-y interpolants of the k+1 coarse planes of the current coarse cell
    T XY[P1][RPT];

    // stage coarse plane zc, interpolate in x (LDS) and y (into XY[pl])
    auto plane = [&](int zc, auto plm) __attribute__((always_inline)) {
        constexpr int pl = decltype(plm)::value;
        const T* __restrict__ src = cs + (long long)zc * NNc;
        for (int i = tid; i < RC * RC; i += NT) {
            const int r = i / RC, c = i - r * RC;
            const int xc = X0c + c, yc = Y0c + r;
            sC[i] = (xc < Nc && yc < Nc) ? src[(long long)yc * Nc + xc] : T(0);
        }
        __syncthreads();
        for (int it = tid; it < RC * TF; it += NT) {
            const int r = it / TF, xf = it - r * TF;
            const int E = xf / J2, j = xf - E * J2;
            const T* pr = &sP[j * P1];
            const T* cr = &sC[r * RC + E * K];
            T v = pr[0] * cr[0];
#pragma unroll
            for (int a = 1; a <= K; ++a) v = fma(pr[a], cr[a], v);
            sXL[r * XP + xf] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int yf = ty + TL::TPY * q;
            T v = T(0);
            if (yf < TF) {
                const int E = yf / J2, j = yf - E * J2;
                const T* pr = &sP[j * P1];
                const T* xr = &sXL[(E * K) * XP + tx];
                v = pr[0] * xr[0];
#pragma unroll
                for (int a = 1; a <= K; ++a) v = fma(pr[a], xr[a * XP], v);
            }
            XY[pl][q] = v;
        }
    };

    // this thread's fine nodes in a plane: 32-bit byte offsets (N^2 sizeof(T) < 2^32)
    const int gx = X0f + tx;
    unsigned roff[RPT];
    unsigned rmask = 0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int yl = ty + TL::TPY * q, gy = Y0f + yl;
        const bool ok = gx < Nf && yl < TF && gy < Nf;
        roff[q] = ok ? ((unsigned)gy * (unsigned)Nf + (unsigned)gx) * (unsigned)sizeof(T) : 0u;
        rmask |= ok ? (1u << q) : 0u;
    }
    for (int E = E0; E < E1; ++E) {
        if (E == E0) plane(E * K, std::integral_constant<int, 0>{});
        tfor<K>([&](auto pm) { plane(E * K + decltype(pm)::value + 1, std::integral_constant<int, decltype(pm)::value + 1>{}); });
        // fine planes 2Ek + j, j = 0..2k-1 (plane 2Ek + 2k is the next cell's
        // j = 0), in two halves of k planes: the old values of a half are all
        // loaded before any of them is written back
        tfor<2>([&](auto hm) {
            constexpr int h = decltype(hm)::value;
            T old[K][RPT];
            tfor<K>([&](auto jm) {
                constexpr int j = h * K + decltype(jm)::value;
                const char* pl = reinterpret_cast<const char*>(fs + (long long)(2 * E * K + j) * NNf);
#pragma unroll
                for (int q = 0; q < RPT; ++q)
                    old[decltype(jm)::value][q] = (rmask >> q & 1u) ? *reinterpret_cast<const T*>(pl + roff[q]) : T(0);
            });
            tfor<K>([&](auto jm) {
                constexpr int j = h * K + decltype(jm)::value;
                char* pl = reinterpret_cast<char*>(fs + (long long)(2 * E * K + j) * NNf);
#pragma unroll
                for (int q = 0; q < RPT; ++q) {
                    if (rmask >> q & 1u) {
                        T v = T(PE<K, j, 0>::v) * XY[0][q];
                        tfor<K>([&](auto am) {
                            constexpr int a = decltype(am)::value + 1;
                            v = fma(T(PE<K, j, a>::v), XY[a][q], v);
                        });
                        *reinterpret_cast<T*>(pl + roff[q]) = old[decltype(jm)::value][q] + v;
                    }
                }
            });
        });
        // the top plane of cell E is the bottom plane of cell E+1
#pragma unroll
        for (int q = 0; q < RPT; ++q) XY[0][q] = XY[K][q];
    }
}

template <int K>
struct RTile {
    static constexpr int CX = (32 / K) > 0 ? (32 / K) : 1;            // coarse cells in x
    static constexpr int TX = CX * K;                                  // coarse nodes in x
    static constexpr int CY0 = 256 / TX > 0 ? 256 / TX : 1;
    static constexpr int CY = CY0 < CX ? CY0 : CX;                     // coarse cells in y
    static constexpr int TY = CY * K;
    static constexpr int NT = TX * CY;                                 // one y-pencil per thread
    static constexpr int FX = 2 * (CX + 1) * K + 1;                    // staged fine width
    static constexpr int FY = 2 * (CY + 1) * K + 1;                    // staged fine height
    static constexpr int XP = TX + 1;
};

// mid[s][zf][yc][xc] = (R_y R_x fine[s][zf])[yc][xc]; grid (tiles, Nf, nstage)
template <int K, typename T>
__global__ void __launch_bounds__(RTile<K>::NT) restrict_xy_kernel(const T* __restrict__ fine, T* __restrict__ mid,
                                                                   int nc, int tiles_x, long long fstride,
                                                                   long long mstride) {
    using TL = RTile<K>;
    constexpr int TX = TL::TX, TY = TL::TY, NT = TL::NT, FX = TL::FX, FY = TL::FY, XP = TL::XP;
    constexpr int CX = TL::CX, J2 = 2 * K;
    __shared__ T sF[FY * FX];
    __shared__ T sR[FY * XP];
    const int Nc = nc * K + 1, Nf = 2 * nc * K + 1;
    const int itx = blockIdx.x % tiles_x, ity = blockIdx.x / tiles_x;
    const int zf = blockIdx.y, s = blockIdx.z;
    const int X0c = itx * TX, Y0c = ity * TY;
    const int FX0 = 2 * X0c - J2, FY0 = 2 * Y0c - J2;     // one coarse cell below the tile
    const int tid = threadIdx.x;
    const T* __restrict__ src = fine + (long long)s * fstride + (long long)zf * Nf * Nf;
    // all loads of the staged region are issued before any LDS write
    constexpr int NS = (FY * FX + NT - 1) / NT;
    T v[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const int i = tid + m * NT;
        const int r = i / FX, c = i - r * FX;
        const int xf = FX0 + c, yf = FY0 + r;
        const bool ok = i < FY * FX && xf >= 0 && xf < Nf && yf >= 0 && yf < Nf;
        v[m] = ok ? src[(long long)yf * Nf + xf] : T(0);
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const int i = tid + m * NT;
        if (m < NS - 1 || i < FY * FX) sF[i] = v[m];
    }
    __syncthreads();
    for (int it = tid; it < FY * CX; it += NT) {
        const int cx = it / FY, r = it - cx * FY;
        T wv[4 * K + 1], o[K];
        const T* row = &sF[r * FX + cx * J2];
#pragma unroll
        for (int u = 0; u <= 4 * K; ++u) wv[u] = row[u];
        rrow<K, T>(wv, o);
#pragma unroll
        for (int a = 0; a < K; ++a) sR[r * XP + cx * K + a] = o[a];
    }
    __syncthreads();
    const int tx = tid % TX, py = tid / TX;
    const int gx = X0c + tx, gy0 = Y0c + py * K;
    if (gx == 0 || gx >= Nc - 1) return;           // boundary columns: zeroed by the z pass
    T wv[4 * K + 1], yv[K];
#pragma unroll
    for (int u = 0; u <= 4 * K; ++u) wv[u] = sR[(py * J2 + u) * XP + tx];
    rrow<K, T>(wv, yv);
    T* dst = mid + (long long)s * mstride + (long long)zf * Nc * Nc;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const int gy = gy0 + a;
        if (gy > 0 && gy < Nc - 1) dst[(long long)gy * Nc + gx] = yv[a];
    }
}

// coarse[s][zc] = R_z mid[s]; grid (ceil(Nc^2 / 256), Nc, nstage)
template <int K, typename T>
__global__ void __launch_bounds__(256) restrict_z_kernel(const T* __restrict__ mid, T* __restrict__ coarse, int nc,
                                                         long long mstride, long long cstride) {
    const int Nc = nc * K + 1;
    const long long NN = (long long)Nc * Nc;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NN) return;
    const int zc = blockIdx.y, s = blockIdx.z;
    T* dst = coarse + (long long)s * cstride + (long long)zc * NN + i;
    const int yc = (int)(i / Nc), xc = (int)(i - (long long)yc * Nc);
    if (zc == 0 || zc == Nc - 1 || xc == 0 || xc == Nc - 1 || yc == 0 || yc == Nc - 1) {
        *dst = T(0);
        return;
    }
    const int E = zc / K, a = zc - E * K;
    const T* m = mid + (long long)s * mstride + i;
    T v = T(0);
    if (a == 0) {
        // cell E-1 (t = 0..2k-1) and cell E (t = 0..2k)
        const T* m0 = m + (long long)(2 * (E - 1) * K) * NN;
        tfor<2 * K>([&](auto tm) {
            constexpr int t = decltype(tm)::value;
            if constexpr (PE<K, t, K>::v != 0.0) v = fma(T(PE<K, t, K>::v), m0[t * NN], v);
        });
        const T* m1 = m + (long long)(2 * E * K) * NN;
        tfor<2 * K + 1>([&](auto tm) {
            constexpr int t = decltype(tm)::value;
            if constexpr (PE<K, t, 0>::v != 0.0) v = fma(T(PE<K, t, 0>::v), m1[t * NN], v);
        });
    } else {
        const T* m1 = m + (long long)(2 * E * K) * NN;
        tfor<K - 1>([&](auto am) {
            constexpr int aa = decltype(am)::value + 1;
            if (a == aa) {
                tfor<2 * K + 1>([&](auto tm) {
                    constexpr int t = decltype(tm)::value;
                    if constexpr (PE<K, t, aa>::v != 0.0) v = fma(T(PE<K, t, aa>::v), m1[t * NN], v);
                });
            }
        });
    }
    *dst = v;
}

template <int K, typename T>
hipError_t restrict_typed(const void* fine, void* coarse, void* tmp, int nc, int nstage, long long fstride,
                          long long cstride, hipStream_t st) {
    using TL = RTile<K>;
    const int Nc = nc * K + 1, Nf = 2 * nc * K + 1;
    const long long mstride = (long long)Nf * Nc * Nc;
    // tiles cover coarse nodes 0 .. Nc-2 (node Nc-1 is boundary)
    const int tiles_x = (Nc - 1 + TL::TX - 1) / TL::TX, tiles_y = (Nc - 1 + TL::TY - 1) / TL::TY;
    restrict_xy_kernel<K, T><<<dim3(tiles_x * tiles_y, Nf, nstage), TL::NT, 0, st>>>(
        static_cast<const T*>(fine), static_cast<T*>(tmp), nc, tiles_x, fstride, mstride);
    const long long NN = (long long)Nc * Nc;
    restrict_z_kernel<K, T><<<dim3((unsigned)((NN + 255) / 256), Nc, nstage), 256, 0, st>>>(
        static_cast<const T*>(tmp), static_cast<T*>(coarse), nc, mstride, cstride);
    return hipGetLastError();
}

template <int K>
hipError_t restrict_k(int dtype, const void* fine, void* coarse, void* tmp, int nc, int nstage,
                      long long fstride, long long cstride, hipStream_t st) {
    return dtype == RK_FP64 ? restrict_typed<K, double>(fine, coarse, tmp, nc, nstage, fstride, cstride, st)
                            : restrict_typed<K, float>(fine, coarse, tmp, nc, nstage, fstride, cstride, st);
}

template <int K, typename T>
hipError_t prolong_typed(const void* coarse, void* fine, int nc, int nstage, long long cstride,
                         long long fstride, hipStream_t st) {
    using TL = PTile<K>;
    ProlongArgs<T> p;
    p.coarse = static_cast<const T*>(coarse);
    p.fine = static_cast<T*>(fine);
    p.cstride = cstride;
    p.fstride = fstride;
    p.nc = nc;
    const int Nf = 2 * nc * K + 1;
    // tiles cover fine nodes 0 .. Nf-2: node Nf-1 is boundary, where the
    // correction is zero
    p.tiles = (Nf - 1 + TL::TF - 1) / TL::TF;
    // coarse cells per z-chunk: enough workgroups to fill the chip
    int czc = 8;
    while (czc > 1 && (long long)p.tiles * p.tiles * ((nc + czc - 1) / czc) * nstage < 2048) czc /= 2;
    p.czc = czc;
    p.chunks = (nc + czc - 1) / czc;
    p.nwork = p.tiles * p.tiles * p.chunks * nstage;
    p.per_xcd = (p.nwork + 7) / 8;
    prolong_add_kernel<K, T><<<8 * p.per_xcd, TL::NT, 0, st>>>(p);
    return hipGetLastError();
}

template <int K>
hipError_t prolong_k(int dtype, const void* coarse, void* fine, int nc, int nstage, long long cstride,
                     long long fstride, hipStream_t st) {
    return dtype == RK_FP64 ? prolong_typed<K, double>(coarse, fine, nc, nstage, cstride, fstride, st)
                            : prolong_typed<K, float>(coarse, fine, nc, nstage, cstride, fstride, st);
}

}  // namespace

hipError_t launch_restrict(int k, int dtype, const void* fine, void* coarse, void* tmp, int nc, int nstage,
                           long long fstride, long long cstride, hipStream_t st) {
    switch (k) {
        case 1: return restrict_k<1>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        case 2: return restrict_k<2>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        case 3: return restrict_k<3>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        case 4: return restrict_k<4>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        case 5: return restrict_k<5>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        case 6: return restrict_k<6>(dtype, fine, coarse, tmp, nc, nstage, fstride, cstride, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_prolong_add(int k, int dtype, const void* coarse, void* fine, int nc, int nstage,
                              long long cstride, long long fstride, hipStream_t st) {
    switch (k) {
        case 1: return prolong_k<1>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        case 2: return prolong_k<2>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        case 3: return prolong_k<3>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        case 4: return prolong_k<4>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        case 5: return prolong_k<5>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        case 6: return prolong_k<6>(dtype, coarse, fine, nc, nstage, cstride, fstride, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk
