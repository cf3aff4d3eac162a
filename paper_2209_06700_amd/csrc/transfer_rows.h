// 1D rows of the multigrid transfers between the n-cell and 2n-cell grids of
// degree k, shared by the transfer kernels and the coarse-level V-cycle kernel.
//
// The prolongation is the embedding of the nested Q_k spaces: within coarse
// cell E the fine nodes 2Ek + j (j = 0..2k) take  sum_a Pe[j][a] x_c[Ek + a]
// (Pe[j][a] = l_a at the fine node).  The restriction is its transpose.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "element_data.h"

namespace rk {
namespace xfer {

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0..N-1.
template <typename F, int... I>
__device__ __forceinline__ void tfor_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void tfor(F&& f) {
    tfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Pe[j][a]: fine node j (0..2k) of a coarse cell, coarse node a (0..k)
template <int K, int J, int A>
struct PE {
    static constexpr double v = elem::Table<K>::d.P[J][A];
};

// Restriction in 1D: out[a], a = 0..k-1, the coarse nodes Ek + a of coarse
// cell E, from w[u] = f(2(E-1)k + u), u = 0..4k.  Coarse node Ek + a collects
//   sum_{t=0}^{2k} Pe[t][a] f(2Ek + t)              (a = 1..k-1), and the vertex
//   a = 0 also  sum_{t=0}^{2k-1} Pe[t][k] f(2(E-1)k + t),
// each fine node counted once (the fine vertex 2Ek has Pe[0][0] = 1).
template <int K, typename T>
__device__ __forceinline__ void rrow(const T* w, T* out) {
    T o = T(PE<K, 0, K>::v) * w[0];
    tfor<2 * K - 1>([&](auto tm) {
        constexpr int t = decltype(tm)::value + 1;
        o = fma(T(PE<K, t, K>::v), w[t], o);
    });
    tfor<2 * K + 1>([&](auto tm) {
        constexpr int t = decltype(tm)::value;
        o = fma(T(PE<K, t, 0>::v), w[2 * K + t], o);
    });
    out[0] = o;
    tfor<K - 1>([&](auto am) {
        constexpr int a = decltype(am)::value + 1;
        T q = T(PE<K, 0, a>::v) * w[2 * K];
        tfor<2 * K>([&](auto tm) {
            constexpr int t = decltype(tm)::value + 1;
            q = fma(T(PE<K, t, a>::v), w[2 * K + t], q);
        });
        out[a] = q;
    });
}

}  // namespace xfer
}  // namespace rk
