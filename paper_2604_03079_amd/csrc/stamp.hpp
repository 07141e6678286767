// Merging a device's local 4x4 matrix onto its node pairs, and writing the merged
// values into A, b (or the hub staging array) through the precomputed stamp codes.
//
// Terminals sharing a node add up: the value of the node pair (a, b) is the left
// fold, in (t, u) row-major order over (d, g, s, b), of the Y entries whose terminal
// nodes are (a, b); RHS rows likewise in terminal order.  Which terminals coincide
// (and which sit on ground) is a "pattern"; each of the 52 possible patterns gets
// its own straight-line code at compile time, and a wave dispatches once per
// distinct pattern among its lanes (one pass for the usual uniform wave).
#pragma once
#include <hip/hip_runtime.h>

#include "kernel_args.hpp"

namespace cs {

// Pattern key: c_t = index of the first terminal on the same node (<= t), or t+1
// for ground; key = c0 + 2*(c1 + 3*(c2 + 4*c3)), 120 codes of which 52 occur.
__device__ __forceinline__ int pattern_key(int t0, int t1, int t2, int t3) {
    const int c0 = t0 == 0 ? 1 : 0;
    const int c1 = t1 == 0 ? 2 : (t1 == t0 ? 0 : 1);
    const int c2 = t2 == 0 ? 3 : (t2 == t0 ? 0 : (t2 == t1 ? 1 : 2));
    const int c3 = t3 == 0 ? 4 : (t3 == t0 ? 0 : (t3 == t1 ? 1 : (t3 == t2 ? 2 : 3)));
    return c0 + 2 * (c1 + 3 * (c2 + 4 * c3));
}

template <int KEY>
struct Pat {
    static constexpr int c(int t) {
        return t == 0 ? KEY % 2 : t == 1 ? (KEY / 2) % 3 : t == 2 ? (KEY / 6) % 4 : (KEY / 24) % 5;
    }
    static constexpr bool ground(int t) { return c(t) == t + 1; }
    static constexpr bool rep(int t) { return c(t) == t; }
    static constexpr bool valid() {
        for (int t = 0; t < 4; ++t)
            if (!ground(t) && !rep(t) && !rep(c(t))) return false;
        return true;
    }
    // compact index of the node of terminal t (-1 for ground)
    static constexpr int idx(int t) {
        if (ground(t)) return -1;
        int a = 0;
        for (int s = 0; s < c(t); ++s)
            if (rep(s)) ++a;
        return a;
    }
    static constexpr int k() {
        int n = 0;
        for (int t = 0; t < 4; ++t)
            if (rep(t)) ++n;
        return n;
    }
};

// Merged value of node pair (a, b).
template <int KEY, int A_, int B_>
__device__ __forceinline__ double merged_entry(const double Y[16]) {
    double m = 0.0;
    bool first = true;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (Pat<KEY>::idx(t) == A_ && Pat<KEY>::idx(u) == B_) {
                m = first ? Y[t * 4 + u] : m + Y[t * 4 + u];
                first = false;
            }
        }
    }
    return m;
}

template <int KEY, int A_>
__device__ __forceinline__ double merged_rhs(const double bl[4]) {
    double m = 0.0;
    bool first = true;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (Pat<KEY>::idx(t) == A_) {
            m = first ? bl[t] : m + bl[t];
            first = false;
        }
    }
    return m;
}

// Merged values of the pattern in code order (k*k matrix entries row-major over
// nodes, then k RHS entries), handed to the sink in one call so that the sink can
// issue all its memory operations back to back.
template <int KEY, int J, class Sink>
__device__ __forceinline__ void put_entry(const double Y[16], const double bl[4], Sink &sink) {
    constexpr int K = Pat<KEY>::k();
    if constexpr (J < K * K) {
        switch (J / K * 4 + J % K) {
#define CS_PE(q) case q: sink.template put<J>(merged_entry<KEY, (q) / 4, (q) % 4>(Y)); break;
            CS_PE(0) CS_PE(1) CS_PE(2) CS_PE(3) CS_PE(4) CS_PE(5) CS_PE(6) CS_PE(7)
            CS_PE(8) CS_PE(9) CS_PE(10) CS_PE(11) CS_PE(12) CS_PE(13) CS_PE(14) CS_PE(15)
#undef CS_PE
            default: break;
        }
    } else {
        constexpr int A = J - K * K;
        sink.template put<J>(merged_rhs<KEY, (A < 4 ? A : 3)>(bl));
    }
}

template <int KEY, int J, int N, class Sink>
__device__ __forceinline__ void put_entries(const double Y[16], const double bl[4], Sink &sink) {
    if constexpr (J < N) {
        put_entry<KEY, J>(Y, bl, sink);
        put_entries<KEY, J + 1, N>(Y, bl, sink);
    }
}

template <int KEY, class Sink>
__device__ __forceinline__ void emit_pattern(const double Y[16], const double bl[4], Sink &sink) {
    if constexpr (Pat<KEY>::valid() && Pat<KEY>::k() > 0 && Sink::kStreaming) {
        // one entry at a time: each merged value is written before the next is formed
        constexpr int K = Pat<KEY>::k();
        put_entries<KEY, 0, K * K + K>(Y, bl, sink);
    } else if constexpr (Pat<KEY>::valid() && Pat<KEY>::k() > 0) {
        constexpr int K = Pat<KEY>::k();
        double m[K * K + K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
#pragma unroll
            for (int b = 0; b < K; ++b) {
                switch (a * 4 + b) {
#define CS_ME(q) case q: m[a * K + b] = merged_entry<KEY, (q) / 4, (q) % 4>(Y); break;
                    CS_ME(0) CS_ME(1) CS_ME(2) CS_ME(3) CS_ME(4) CS_ME(5) CS_ME(6) CS_ME(7)
                    CS_ME(8) CS_ME(9) CS_ME(10) CS_ME(11) CS_ME(12) CS_ME(13) CS_ME(14) CS_ME(15)
#undef CS_ME
                    default: break;
                }
            }
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            switch (a) {
                case 0: m[K * K + a] = merged_rhs<KEY, 0>(bl); break;
                case 1: m[K * K + a] = merged_rhs<KEY, 1>(bl); break;
                case 2: m[K * K + a] = merged_rhs<KEY, 2>(bl); break;
                default: m[K * K + a] = merged_rhs<KEY, 3>(bl); break;
            }
        }
        sink.template stamp<K * K, K>(m);
    }
}

// Uniform-key dispatch (key must be wave-uniform).
template <class Sink>
__device__ __forceinline__ void emit_uniform(int key, const double Y[16], const double bl[4],
                                             Sink &sink) {
    switch (key) {
#define CS_K(q) case q: emit_pattern<q>(Y, bl, sink); break;
#define CS_K10(q) CS_K(q) CS_K(q + 1) CS_K(q + 2) CS_K(q + 3) CS_K(q + 4) CS_K(q + 5) \
    CS_K(q + 6) CS_K(q + 7) CS_K(q + 8) CS_K(q + 9)
        CS_K10(0) CS_K10(10) CS_K10(20) CS_K10(30) CS_K10(40) CS_K10(50)
        CS_K10(60) CS_K10(70) CS_K10(80) CS_K10(90) CS_K10(100) CS_K10(110)
#undef CS_K10
#undef CS_K
        default: break;
    }
}

// Per-lane key: one pass per distinct key present among the active lanes.
template <class Sink>
__device__ __forceinline__ void emit_merged(int key, const double Y[16], const double bl[4],
                                            Sink &sink) {
    for (;;) {
        const int k0 = __builtin_amdgcn_readfirstlane(key);
        if (key == k0) {
            emit_uniform(k0, Y, bl, sink);
            break;
        }
    }
}

// Coloured stamping: tag STORE writes, tag ADD loads and adds, tag HUB stages.
// -0.0 is the exact identity of IEEE addition, so "store" is "-0.0 + value".
// COHERENT: the accesses are agent-scope relaxed atomics (coherent across the
// XCDs' separate L2 caches), so a later colour phase in the same persistent
// kernel reads what an earlier phase wrote on another XCD without any L2
// write-back or invalidation; ordering comes from the grid barrier.  All loads of
// a device are issued before its first store (its entries are distinct).
template <bool COHERENT>
struct ColourSinkT {
    static constexpr bool kStreaming = false;
    const int32_t *code;
    int32_t n, pos;
    double *A, *b, *stage;
    template <int NA, int NB>
    __device__ __forceinline__ void stamp(const double *m) {
        constexpr int N = NA + NB;
        double *p[N];
        double old[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const uint32_t c = (uint32_t)code[(size_t)j * n + pos];
            const uint32_t tag = c >> 30;
            const uint32_t idx = c & 0x3FFFFFFFu;
            p[j] = tag == TAG_HUB ? stage + idx : (j >= NA ? b : A) + idx;
            old[j] = -0.0;
            if (tag == TAG_ADD) {
                if constexpr (COHERENT) old[j] = __hip_atomic_load(p[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else old[j] = *p[j];
            }
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if constexpr (COHERENT) __hip_atomic_store(p[j], old[j] + m[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else *p[j] = old[j] + m[j];
        }
    }
};
using ColourSink = ColourSinkT<false>;

// Atomic stamping: every entry (hub entries included) is an FP64 atomic add.
struct AtomicSink {
    static constexpr bool kStreaming = false;
    const int32_t *acode;
    int32_t n, pos;
    double *A, *b;
    template <int NA, int NB>
    __device__ __forceinline__ void stamp(const double *m) {
#pragma unroll
        for (int j = 0; j < NA + NB; ++j) {
            const int32_t idx = acode[(size_t)j * n + pos];
            (void)unsafeAtomicAdd((j >= NA ? b : A) + idx, m[j]);
        }
    }
};

// Atomic stamping with hub entries held back: an entry whose colour code marks it a
// hub (a rail entry every device on that rail writes) is recorded in the lane (up to
// HS of them, the rest added at once); the kernel then sums each hub target over the
// wave and adds the sum with one atomic, so the rails take one atomic per wave
// instead of one per device.
template <int HS>
struct AtomicHubSink {
    static constexpr bool kStreaming = false;
    const int32_t *acode;
    const int32_t *code;
    int32_t n, pos;
    double *A, *b;
    int nh = 0;
    int32_t tgt[HS];   // A index, or b row | HUB_B_FLAG
    double val[HS];
    template <int NA, int NB>
    __device__ __forceinline__ void stamp(const double *m) {
#pragma unroll
        for (int j = 0; j < NA + NB; ++j) {
            const int32_t idx = acode[(size_t)j * n + pos];
            const bool hub = ((uint32_t)code[(size_t)j * n + pos] >> 30) == TAG_HUB;
            if (hub && nh < HS) {
                const int32_t t = j >= NA ? (int32_t)((uint32_t)idx | HUB_B_FLAG) : idx;
#pragma unroll
                for (int s = 0; s < HS; ++s)
                    if (s == nh) {
                        tgt[s] = t;
                        val[s] = m[j];
                    }
                ++nh;
            } else {
                (void)unsafeAtomicAdd((j >= NA ? b : A) + idx, m[j]);
            }
        }
    }
};

// LDS row sink (region schedule): merged value j of a lane goes to p[j * stride].
struct LdsRowSink {
    static constexpr bool kStreaming = true;
    double *p;
    int stride;
    template <int J>
    __device__ __forceinline__ void put(double v) {
        p[J * stride] = v;
    }
};

// The same, keeping a copy of each merged value in r[J] (a local array the caller
// indexes with constants only, so that it lives in registers).
struct LdsRowRegSink {
    static constexpr bool kStreaming = true;
    double *p;
    int stride;
    double *r;
    template <int J>
    __device__ __forceinline__ void put(double v) {
        p[J * stride] = v;
        r[J] = v;
    }
};

// Buffer sink: merged values into a [NCODE][n] buffer (the buffered variant).
struct BufferSink {
    static constexpr bool kStreaming = false;
    double *buf;
    int32_t n, pos;
    template <int NA, int NB>
    __device__ __forceinline__ void stamp(const double *m) {
#pragma unroll
        for (int j = 0; j < NA + NB; ++j) buf[(size_t)j * n + pos] = m[j];
    }
};

}  // namespace cs
