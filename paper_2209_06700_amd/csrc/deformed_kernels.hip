// Cell-based operator on a deformed (non-affine) hexahedral mesh.
//
// The mesh is the uniform n^3 mesh of the unit cube mapped by
//   Phi(x) = x + eps s(x) (1,1,1),  s(x) = sin(pi x1) sin(pi x2) sin(pi x3),
// with Q_k elements on the reference cell (Gauss-Lobatto nodes) and the
// (k+1)^3-point Gauss rule.  On such a mesh the element matrices differ from
// cell to cell, so the operator evaluates cell integrals by sum factorisation
// with per-point geometry: per Gauss point the mass factor m = w det J and the
// symmetric stiffness metric G = w det J J^-1 J^-T (7 values).  Sec. 3.4
// names this data as the reason to batch stages: the kernel loads a cell's
// geometry once and applies it to all Q stages of the launch.
//
// Work decomposition: a workgroup owns CPW = 256 / (k+1)^2 cells of one
// colour (cells whose index parity equals the colour bits), (k+1)^2 threads
// per cell.  Cells of one colour share no node, so the eight colour launches
// accumulate into the output without atomics and in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "element_data.h"
#include "rk_internal.h"

namespace rk {
namespace {

constexpr int kGeo = 7;   // m, Gxx, Gyy, Gzz, Gxy, Gxz, Gyz

// Gauss point / weight q of degree K's rule (runtime q selects a constant)
template <int K>
__device__ __forceinline__ double gauss_x(int q) {
    double r = 0.0;
#pragma unroll
    for (int t = 0; t <= K; ++t)
        if (t == q) r = elem::Table<K>::d.gx[t];
    return r;
}
template <int K>
__device__ __forceinline__ double gauss_w(int q) {
    double r = 0.0;
#pragma unroll
    for (int t = 0; t <= K; ++t)
        if (t == q) r = elem::Table<K>::d.gw[t];
    return r;
}

template <int K, typename T>
__global__ void __launch_bounds__(256) geometry_kernel(T* __restrict__ geo, int n, double eps) {
    constexpr int NQ = K + 1, NP = NQ * NQ * NQ;
    const long long total = (long long)n * n * n * NP;
    const double h = 1.0 / n, pi = 3.14159265358979323846;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long cell = t / NP;
        const int q = (int)(t - cell * NP);
        const int qa = q % NQ, qb = (q / NQ) % NQ, qc = q / (NQ * NQ);
        const int cx = (int)(cell % n), cy = (int)((cell / n) % n), cz = (int)(cell / ((long long)n * n));
        double x[3] = {h * (cx + gauss_x<K>(qa)), h * (cy + gauss_x<K>(qb)), h * (cz + gauss_x<K>(qc))};
        double sn[3], cs[3];
        for (int d = 0; d < 3; ++d) { sn[d] = sin(pi * x[d]); cs[d] = cos(pi * x[d]); }
        // grad s; Phi' = I + eps (1,1,1)^T grad s^T
        const double g[3] = {pi * cs[0] * sn[1] * sn[2], pi * sn[0] * cs[1] * sn[2], pi * sn[0] * sn[1] * cs[2]};
        const double a = 1.0 + eps * (g[0] + g[1] + g[2]);      // det Phi'
        // Phi'^-1 = I - eps (1,1,1)^T grad s^T / a (Sherman-Morrison); J = h Phi'
        double Ji[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Ji[r][c] = ((r == c ? 1.0 : 0.0) - eps * g[c] / a) / h;
        const double w = gauss_w<K>(qa) * gauss_w<K>(qb) * gauss_w<K>(qc);
        const double wdet = w * a * h * h * h;
        double C[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) C[r][c] = Ji[r][0] * Ji[c][0] + Ji[r][1] * Ji[c][1] + Ji[r][2] * Ji[c][2];
        T* o = geo + cell * (long long)(kGeo * NP) + q;
        o[0 * NP] = T(wdet);
        o[1 * NP] = T(wdet * C[0][0]);
        o[2 * NP] = T(wdet * C[1][1]);
        o[3 * NP] = T(wdet * C[2][2]);
        o[4 * NP] = T(wdet * C[0][1]);
        o[5 * NP] = T(wdet * C[0][2]);
        o[6 * NP] = T(wdet * C[1][2]);
    }
}

template <typename T>
struct DefArgs {
    const T* u;                // stiffness-term input (and mass-term input unless PAIR)
    const T* um;               // PAIR: mass-term input
    T* v;
    const T* geo;
    long long stride;          // N^3
    int n, nstage;
    int bx, by, bz;            // colour bits
    int ccx, ccy, ccz;         // cells of this colour per direction
    long long ncell;           // ccx ccy ccz
    T alpha[RK_MAX_Q], beta[RK_MAX_Q];
};

// Each one-dimensional contraction runs along pencils of its own direction:
// the N2 = (k+1)^2 threads of a cell take the pencils along z (thread (a, b)
// = (x, y)), along y ((a, b) = (x, z)) or along x ((a, b) = (y, z)), so every
// coefficient of the 1D tables is a compile-time constant and a pass moves
// k+1 values per thread through LDS.  Cell arrays in LDS are [z][y][x].
// PAIR: v_s = alpha_s M um_s + beta_s K u_s (two inputs, as in the stage
// operator of eq. irk:A with a pre-mixed mass-term input).
template <int K, typename T, bool PAIR>
__global__ void __launch_bounds__(256) deformed_op_kernel(DefArgs<T> p) {
    constexpr auto& E = elem::Table<K>::d;
    constexpr int NQ = K + 1, N2 = NQ * NQ, NP = N2 * NQ;
    constexpr int CPW = 256 / N2;
    __shared__ T L0[CPW * NP];
    __shared__ T L1[CPW * NP];
    __shared__ T L2[CPW * NP];
    const int tid = threadIdx.x;
    const int lc = tid / N2;
    const bool lane = lc < CPW;                      // owns an LDS slot
    const int r = tid - lc * N2;
    const int a = r % NQ, b = r / NQ;
    const long long cid = (long long)blockIdx.x * CPW + lc;
    const bool valid = lane && cid < p.ncell;
    int cx = 0, cy = 0, cz = 0;
    if (valid) {
        cx = 2 * (int)(cid % p.ccx) + p.bx;
        cy = 2 * (int)((cid / p.ccx) % p.ccy) + p.by;
        cz = 2 * (int)(cid / ((long long)p.ccx * p.ccy)) + p.bz;
    }
    const int n = p.n, N = n * K + 1;
    const long long NN = (long long)N * N;
    T* A = L0 + (lane ? lc : 0) * NP;
    T* B = L1 + (lane ? lc : 0) * NP;
    T* C = L2 + (lane ? lc : 0) * NP;
    const int zb = a + NQ * b;          // z pencil (x = a, y = b): element zb + N2 l
    const int yb = a + N2 * b;          // y pencil (x = a, z = b): element yb + NQ m
    const int xb = NQ * a + N2 * b;     // x pencil (y = a, z = b): element xb + m
    // geometry of this thread's z pencil of points, loaded once for all stages
    T gm[kGeo][NQ];
    {
        const long long cell = (long long)cx + (long long)n * (cy + (long long)n * cz);
        const T* g = p.geo + cell * (long long)(kGeo * NP) + zb;
#pragma unroll
        for (int c = 0; c < kGeo; ++c)
#pragma unroll
            for (int q = 0; q < NQ; ++q) gm[c][q] = valid ? g[c * NP + q * N2] : T(0);
    }
    // node (cx K + a, cy K + b, cz K + l) of the z pencil
    const int gxn = cx * K + a, gyn = cy * K + b, gz0 = cz * K;
    const bool col_in = valid && gxn > 0 && gxn < N - 1 && gyn > 0 && gyn < N - 1;
    const long long colbase = (long long)gyn * N + gxn;
    // Software pipeline over the stages: the input pencils of stage s+1 are
    // loaded while stage s runs its passes, and the output values that the
    // accumulation of stage s adds to are loaded when the stage starts (no
    // other cell of this colour touches these nodes), so that neither waits
    // for memory between two barriers.
    auto nodal = [&](const T* base, int l) __attribute__((always_inline)) {
        const int z = gz0 + l;
        return (col_in && z > 0 && z < N - 1) ? base[colbase + z * NN] : T(0);
    };
    T nu[NQ], num[PAIR ? NQ : 1];
#pragma unroll
    for (int l = 0; l < NQ; ++l) {
        nu[l] = nodal(p.u, l);
        if constexpr (PAIR) num[l] = nodal(p.um, l);
    }
    for (int s = 0; s < p.nstage; ++s) {
        T v[NQ], w[NQ];
        T UM[NQ];   // PAIR: the mass-term input at this z pencil of points
        T cu[NQ], vo[NQ];
        T* vs = p.v + (long long)s * p.stride;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            cu[l] = nu[l];
            if constexpr (PAIR) v[l] = num[l];
            vo[l] = nodal(vs, l);
        }
        if (s + 1 < p.nstage) {
#pragma unroll
            for (int l = 0; l < NQ; ++l) {
                nu[l] = nodal(p.u + (long long)(s + 1) * p.stride, l);
                if constexpr (PAIR) num[l] = nodal(p.um + (long long)(s + 1) * p.stride, l);
            }
        }
        if constexpr (PAIR) {
            if (lane)
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    T acc = T(0);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                    A[zb + N2 * q] = acc;
                }
            __syncthreads();
            if (lane) {
#pragma unroll
                for (int m = 0; m < NQ; ++m) v[m] = A[yb + NQ * m];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    T acc = T(0);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                    B[yb + NQ * q] = acc;
                }
            }
            __syncthreads();
            if (lane) {
#pragma unroll
                for (int m = 0; m < NQ; ++m) v[m] = B[xb + m];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    T acc = T(0);
#pragma unroll
                    for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                    C[xb + q] = acc;
                }
            }
            __syncthreads();
            if (lane)
#pragma unroll
                for (int q = 0; q < NQ; ++q) UM[q] = C[zb + N2 * q];
            // A, B are free (their reads are behind the last barrier); C is
            // rewritten only after the next two barriers
        }
#pragma unroll
        for (int l = 0; l < NQ; ++l) v[l] = cu[l];
        // values at the Gauss points: z, y, x
        if (lane)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T acc = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                A[zb + N2 * q] = acc;
            }
        __syncthreads();
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) v[m] = A[yb + NQ * m];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T acc = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                B[yb + NQ * q] = acc;
            }
        }
        __syncthreads();
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) v[m] = B[xb + m];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T acc = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc = fma(T(E.gB[q][m]), v[m], acc);
                A[xb + q] = acc;
            }
        }
        __syncthreads();
        // reference derivatives along y (into B) and x (into C), collocation
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) { v[m] = A[yb + NQ * m]; w[m] = A[xb + m]; }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T dy = T(0), dx = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    dy = fma(T(E.gD[q][m]), v[m], dy);
                    dx = fma(T(E.gD[q][m]), w[m], dx);
                }
                B[yb + NQ * q] = dy;
                C[xb + q] = dx;
            }
        }
        __syncthreads();
        // the point operation on z pencils, with the z derivative and its
        // transpose in registers
        if (lane) {
            T U[NQ], dy[NQ], dx[NQ], fz[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) { U[q] = A[zb + N2 * q]; dy[q] = B[zb + N2 * q]; dx[q] = C[zb + N2 * q]; }
            const T al = p.alpha[s], be = p.beta[s];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T dz = T(0);
#pragma unroll
                for (int m = 0; m < NQ; ++m) dz = fma(T(E.gD[q][m]), U[m], dz);
                v[q] = al * gm[0][q] * (PAIR ? UM[q] : U[q]);
                const T fx = be * (gm[1][q] * dx[q] + gm[4][q] * dy[q] + gm[5][q] * dz);
                const T fy = be * (gm[4][q] * dx[q] + gm[2][q] * dy[q] + gm[6][q] * dz);
                fz[q] = be * (gm[5][q] * dx[q] + gm[6][q] * dy[q] + gm[3][q] * dz);
                B[zb + N2 * q] = fy;
                C[zb + N2 * q] = fx;
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T acc = v[q];
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc = fma(T(E.gD[m][q]), fz[m], acc);
                A[zb + N2 * q] = acc;
            }
        }
        __syncthreads();
        // transposed y derivative, added on y pencils
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) v[m] = B[yb + NQ * m];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                T acc = A[yb + NQ * q];
#pragma unroll
                for (int m = 0; m < NQ; ++m) acc = fma(T(E.gD[m][q]), v[m], acc);
                A[yb + NQ * q] = acc;
            }
        }
        __syncthreads();
        // transposed x derivative, then back to the x nodes, on x pencils
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) { v[m] = C[xb + m]; w[m] = A[xb + m]; }
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int m = 0; m < NQ; ++m) w[q] = fma(T(E.gD[m][q]), v[m], w[q]);
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc = fma(T(E.gB[q][i]), w[q], acc);
                B[xb + i] = acc;
            }
        }
        __syncthreads();
        // back to the y nodes on y pencils
        if (lane) {
#pragma unroll
            for (int m = 0; m < NQ; ++m) v[m] = B[yb + NQ * m];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc = fma(T(E.gB[q][j]), v[q], acc);
                C[yb + NQ * j] = acc;
            }
        }
        __syncthreads();
        // back to the z nodes on z pencils, accumulated into v
        if (lane) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) w[q] = C[zb + N2 * q];
#pragma unroll
            for (int l = 0; l < NQ; ++l) {
                T acc = T(0);
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc = fma(T(E.gB[q][l]), w[q], acc);
                const int z = gz0 + l;
                if (col_in && z > 0 && z < N - 1) vs[colbase + z * NN] = vo[l] + acc;
            }
        }
    }
}

// Jacobi diagonals of the deformed-mesh M and K: per cell of one colour and
// node (a, b, c) of the cell,
//   diag M += sum_q m_q  B_a^2 B_b^2 B_c^2,
//   diag K += sum_q grad(phi)^T G_q grad(phi) with grad(phi) = (D_a B_b B_c,
//             B_a D_b B_c, B_a B_b D_c) at point q,
// B = gB, D = gBd (values and derivatives of the GLL basis at the Gauss
// points).  One thread per node, the cell's geometry staged in LDS.
template <int K, typename T>
__global__ void __launch_bounds__(512) deformed_diag_kernel(const T* __restrict__ geo, T* __restrict__ dM,
                                                            T* __restrict__ dK, int n, int bx, int by, int bz,
                                                            int ccx, int ccy, long long ncell) {
    constexpr auto& E = elem::Table<K>::d;
    constexpr int NQ = K + 1, N2 = NQ * NQ, NP = N2 * NQ;
    constexpr int CPW = 512 / NP;
    __shared__ T sg[CPW * kGeo * NP];
    const int tid = threadIdx.x;
    const int lc = tid / NP;
    const bool lane = lc < CPW;
    const int r = tid - lc * NP;
    const int a = r % NQ, b = (r / NQ) % NQ, c = r / N2;
    const long long cid = (long long)blockIdx.x * CPW + lc;
    const bool valid = lane && cid < ncell;
    int cx = 0, cy = 0, cz = 0;
    if (valid) {
        cx = 2 * (int)(cid % ccx) + bx;
        cy = 2 * (int)((cid / ccx) % ccy) + by;
        cz = 2 * (int)(cid / ((long long)ccx * ccy)) + bz;
    }
    const long long cell = (long long)cx + (long long)n * (cy + (long long)n * cz);
    if (lane)
        for (int i = r; i < kGeo * NP; i += NP) sg[lc * kGeo * NP + i] = valid ? geo[cell * (kGeo * NP) + i] : T(0);
    __syncthreads();
    if (!valid) return;
    // squares and products of the 1D values at this node's a, b, c
    T Ba[NQ], Da[NQ], Bb[NQ], Db[NQ], Bc[NQ], Dc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Ba[q] = Da[q] = Bb[q] = Db[q] = Bc[q] = Dc[q] = T(0);
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            if (t == a) { Ba[q] = T(E.gB[q][t]); Da[q] = T(E.gBd[q][t]); }
            if (t == b) { Bb[q] = T(E.gB[q][t]); Db[q] = T(E.gBd[q][t]); }
            if (t == c) { Bc[q] = T(E.gB[q][t]); Dc[q] = T(E.gBd[q][t]); }
        }
    }
    const T* g = sg + lc * kGeo * NP;
    T dm = T(0), dk = T(0);
#pragma unroll
    for (int qz = 0; qz < NQ; ++qz)
#pragma unroll
        for (int qy = 0; qy < NQ; ++qy)
#pragma unroll
            for (int qx = 0; qx < NQ; ++qx) {
                const int q = qx + NQ * (qy + NQ * qz);
                const T v = Ba[qx] * Bb[qy] * Bc[qz];
                const T gx = Da[qx] * Bb[qy] * Bc[qz], gy = Ba[qx] * Db[qy] * Bc[qz], gz = Ba[qx] * Bb[qy] * Dc[qz];
                dm = fma(g[q] * v, v, dm);
                const T fx = g[1 * NP + q] * gx + g[4 * NP + q] * gy + g[5 * NP + q] * gz;
                const T fy = g[4 * NP + q] * gx + g[2 * NP + q] * gy + g[6 * NP + q] * gz;
                const T fz = g[5 * NP + q] * gx + g[6 * NP + q] * gy + g[3 * NP + q] * gz;
                dk = fma(fx, gx, fma(fy, gy, fma(fz, gz, dk)));
            }
    const int N = n * K + 1;
    const int ix = cx * K + a, iy = cy * K + b, iz = cz * K + c;
    if (ix > 0 && ix < N - 1 && iy > 0 && iy < N - 1 && iz > 0 && iz < N - 1) {
        const long long node = (long long)ix + (long long)N * (iy + (long long)N * iz);
        dM[node] += dm;
        dK[node] += dk;
    }
}

template <int K, typename T>
hipError_t diag_typed(int n, const void* geo, void* dM, void* dK, hipStream_t st) {
    constexpr int NP = (K + 1) * (K + 1) * (K + 1), CPW = 512 / NP;
    const long long N = (long long)n * K + 1;
    const int dt = sizeof(T) == 8 ? RK_FP64 : RK_FP32;
    hipError_t e = launch_fill(dt, dM, N * N * N, 0.0, st);
    if (e == hipSuccess) e = launch_fill(dt, dK, N * N * N, 0.0, st);
    for (int colour = 0; colour < 8 && e == hipSuccess; ++colour) {
        const int bx = colour & 1, by = (colour >> 1) & 1, bz = (colour >> 2) & 1;
        const int ccx = (n - bx + 1) / 2, ccy = (n - by + 1) / 2, ccz = (n - bz + 1) / 2;
        const long long ncell = (long long)ccx * ccy * ccz;
        if (ncell == 0) continue;
        deformed_diag_kernel<K, T><<<dim3((unsigned)((ncell + CPW - 1) / CPW)), dim3(512), 0, st>>>(
            static_cast<const T*>(geo), static_cast<T*>(dM), static_cast<T*>(dK), n, bx, by, bz, ccx, ccy, ncell);
        e = hipGetLastError();
    }
    return e;
}

// Streaming Chebyshev pieces with stored diagonals: D_s = alpha_s dM + beta_s dK.
struct VecScal {
    double alpha[RK_MAX_Q], beta[RK_MAX_Q];
};

// x_new = x + ca (x - xo) + cb D^-1 (b - t) on interior nodes (xo null: 0;
// x null: 0), 0 on boundary nodes; x_new may alias x or xo.  Stages
// [0, nstage) of vectors with stage stride N^3.
template <typename T>
__global__ void __launch_bounds__(256) cheb_vec_kernel(T* xn, const T* x, const T* xo, const T* __restrict__ b,
                                                       const T* __restrict__ t, const T* __restrict__ dM,
                                                       const T* __restrict__ dK, VecScal sc, double ca, double cb,
                                                       int N, int nstage) {
    const long long N3 = (long long)N * N * N;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < N3 * nstage;
         idx += (long long)gridDim.x * blockDim.x) {
        const int s = (int)(idx / N3);
        const long long r = idx - s * N3;
        const int z = (int)(r / ((long long)N * N));
        const int rr = (int)(r - (long long)z * N * N);
        const int y = rr / N, xx = rr - y * N;
        T out = T(0);
        if (xx > 0 && xx < N - 1 && y > 0 && y < N - 1 && z > 0 && z < N - 1) {
            const T D = T(sc.alpha[s]) * dM[r] + T(sc.beta[s]) * dK[r];
            const T xv = x ? x[idx] : T(0);
            const T xov = xo ? xo[idx] : T(0);
            const T tv = t ? t[idx] : T(0);
            out = xv + T(ca) * (xv - xov) + T(cb) * (b[idx] - tv) / D;
        }
        xn[idx] = out;
    }
}

// v = b - v (the residual after an operator application), any type
template <typename T>
__global__ void __launch_bounds__(256) resid_vec_kernel(T* v, const T* __restrict__ b, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        v[i] = b[i] - v[i];
}

template <int K, typename T>
hipError_t launch_typed(int n, int Q, const double* alpha, const double* beta, const void* geo,
                        const void* um, const void* u, void* v, hipStream_t st) {
    constexpr int NQ = K + 1, N2 = NQ * NQ, CPW = 256 / N2;
    const long long N = (long long)n * K + 1;
    DefArgs<T> a;
    a.u = static_cast<const T*>(u);
    a.um = static_cast<const T*>(um);
    a.v = static_cast<T*>(v);
    a.geo = static_cast<const T*>(geo);
    a.stride = N * N * N;
    a.n = n;
    a.nstage = Q;
    for (int s = 0; s < RK_MAX_Q; ++s) {
        a.alpha[s] = T(s < Q ? alpha[s] : 0.0);
        a.beta[s] = T(s < Q ? beta[s] : 0.0);
    }
    hipError_t e = launch_fill(sizeof(T) == 8 ? RK_FP64 : RK_FP32, v, (long long)Q * a.stride, 0.0, st);
    if (e != hipSuccess) return e;
    for (int colour = 0; colour < 8; ++colour) {
        a.bx = colour & 1;
        a.by = (colour >> 1) & 1;
        a.bz = (colour >> 2) & 1;
        a.ccx = (n - a.bx + 1) / 2;
        a.ccy = (n - a.by + 1) / 2;
        a.ccz = (n - a.bz + 1) / 2;
        a.ncell = (long long)a.ccx * a.ccy * a.ccz;
        if (a.ncell == 0) continue;
        const long long blocks = (a.ncell + CPW - 1) / CPW;
        if (um != u) deformed_op_kernel<K, T, true><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(a);
        else deformed_op_kernel<K, T, false><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int K, typename T>
hipError_t geometry_typed(int n, double eps, void* geo, hipStream_t st) {
    constexpr int NP = (K + 1) * (K + 1) * (K + 1);
    const long long total = (long long)n * n * n * NP;
    const long long blocks = std::min<long long>((total + 255) / 256, 1 << 20);
    geometry_kernel<K, T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(static_cast<T*>(geo), n, eps);
    return hipGetLastError();
}

}  // namespace

size_t deformed_geometry_elems(int n, int k) {
    return (size_t)n * n * n * kGeo * (size_t)(k + 1) * (k + 1) * (k + 1);
}

hipError_t launch_deformed_geometry(int k, int dtype, int n, double eps, void* geo, hipStream_t st) {
#define RK_DEF_GEO(KK)                                                                         \
    case KK:                                                                                   \
        return dtype == RK_FP64 ? geometry_typed<KK, double>(n, eps, geo, st)                  \
                                : geometry_typed<KK, float>(n, eps, geo, st);
    switch (k) {
        RK_DEF_GEO(1) RK_DEF_GEO(2) RK_DEF_GEO(3) RK_DEF_GEO(4) RK_DEF_GEO(5) RK_DEF_GEO(6)
        default: return hipErrorInvalidValue;
    }
#undef RK_DEF_GEO
}

hipError_t launch_deformed_diag(int k, int dtype, int n, const void* geo, void* dM, void* dK, hipStream_t st) {
#define RK_DEF_DIAG(KK)                                                                    \
    case KK:                                                                               \
        return dtype == RK_FP64 ? diag_typed<KK, double>(n, geo, dM, dK, st)               \
                                : diag_typed<KK, float>(n, geo, dM, dK, st);
    switch (k) {
        RK_DEF_DIAG(1) RK_DEF_DIAG(2) RK_DEF_DIAG(3) RK_DEF_DIAG(4) RK_DEF_DIAG(5) RK_DEF_DIAG(6)
        default: return hipErrorInvalidValue;
    }
#undef RK_DEF_DIAG
}

hipError_t launch_cheb_vec(int dtype, void* xn, const void* x, const void* xo, const void* b, const void* t,
                           const void* dM, const void* dK, const double* alpha, const double* beta, double ca,
                           double cb, int N, int nstage, hipStream_t st) {
    VecScal sc{};
    for (int s = 0; s < nstage && s < RK_MAX_Q; ++s) { sc.alpha[s] = alpha[s]; sc.beta[s] = beta[s]; }
    const long long total = (long long)N * N * N * nstage;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 1 << 16);
    if (dtype == RK_FP64)
        cheb_vec_kernel<double><<<blocks, 256, 0, st>>>((double*)xn, (const double*)x, (const double*)xo,
                                                        (const double*)b, (const double*)t, (const double*)dM,
                                                        (const double*)dK, sc, ca, cb, N, nstage);
    else
        cheb_vec_kernel<float><<<blocks, 256, 0, st>>>((float*)xn, (const float*)x, (const float*)xo,
                                                       (const float*)b, (const float*)t, (const float*)dM,
                                                       (const float*)dK, sc, ca, cb, N, nstage);
    return hipGetLastError();
}

hipError_t launch_resid_vec(int dtype, void* v, const void* b, long long n, hipStream_t st) {
    const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 1 << 16);
    if (dtype == RK_FP64) resid_vec_kernel<double><<<blocks, 256, 0, st>>>((double*)v, (const double*)b, n);
    else resid_vec_kernel<float><<<blocks, 256, 0, st>>>((float*)v, (const float*)b, n);
    return hipGetLastError();
}

hipError_t launch_deformed_apply(int k, int dtype, int n, int Q, const double* alpha, const double* beta,
                                 const void* geo, const void* um, const void* u, void* v, hipStream_t st) {
#define RK_DEF_OP(KK)                                                                              \
    case KK:                                                                                       \
        return dtype == RK_FP64 ? launch_typed<KK, double>(n, Q, alpha, beta, geo, um, u, v, st)   \
                                : launch_typed<KK, float>(n, Q, alpha, beta, geo, um, u, v, st);
    switch (k) {
        RK_DEF_OP(1) RK_DEF_OP(2) RK_DEF_OP(3) RK_DEF_OP(4) RK_DEF_OP(5) RK_DEF_OP(6)
        default: return hipErrorInvalidValue;
    }
#undef RK_DEF_OP
}

}  // namespace rk
