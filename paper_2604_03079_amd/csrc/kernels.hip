// HIP kernels for gfx950: the region schedule of the coloured fused
// evaluate-and-stamp (one workgroup per region, and its grid-barrier form), the
// persistent colour-phase kernel, one-kernel-per-colour, buffered-colour,
// serial-stamp and atomic variants, and the hub reduction.  The adjoint kernel is in
// adjoint.hip.
//
// Paper, Methodology: colours are processed sequentially; within a colour every
// device is evaluated and stamped in parallel, no two of them touching the same
// entry, so stamping needs neither locks nor atomics.  Table "Summary of BSIM4
// evaluation-kernel variants" lists the schedules mirrored here.
#include <hip/hip_runtime.h>

#include "kernel_args.hpp"
#include "launch.hpp"
#include "model.hpp"
#include "stamp.hpp"

namespace cs {

// ---- per-device helpers -----------------------------------------------------------

struct DevIn {
    int32_t t0, t1, t2, t3;
    int key;
};

// Element pos of a per-position table row that starts at row (the same address on
// every lane): a uniform base plus a 32-bit byte offset, the form the global loads
// take directly, so a row costs no per-lane 64-bit address arithmetic.  Positions
// are below 2^31 / NCODE (checked when a circuit or batch is created), so the
// offset of an 8-byte element fits 32 bits.
static_assert(NCODE >= 8, "a position's byte offset in an 8-byte row fits 32 bits");
template <class T>
__device__ __forceinline__ T ld_row(const T *row, int pos) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + (uint32_t)pos * (uint32_t)sizeof(T));
}

__device__ __forceinline__ DevIn load_terms(const KCirc &kc, int pos) {
    DevIn d;
    const size_t n = (size_t)kc.n;
    d.t0 = ld_row(kc.term, pos);
    d.t1 = ld_row(kc.term + n, pos);
    d.t2 = ld_row(kc.term + 2 * n, pos);
    d.t3 = ld_row(kc.term + 3 * n, pos);
    d.key = pattern_key(d.t0, d.t1, d.t2, d.t3);
    return d;
}

__device__ __forceinline__ double volt(const double *x, int32_t t) { return t == 0 ? 0.0 : x[t - 1]; }

// Per-device constants of position pos (rows of kc.sdp; the junction area only
// when the junction terms are compiled in).
template <bool J>
__device__ __forceinline__ DevConstT<double> load_consts(const KCirc &kc, int pos) {
    const size_t n = (size_t)kc.n;
    DevConstT<double> k;
    k.vth_s = ld_row(kc.sdp, pos);
    k.dibl = ld_row(kc.sdp + n, pos);
    k.nsce = ld_row(kc.sdp + 2 * n, pos);
    k.beta0 = ld_row(kc.sdp + 3 * n, pos);
    k.lambda = ld_row(kc.sdp + 4 * n, pos);
    k.k1AbL = ld_row(kc.sdp + 5 * n, pos);
    k.esatn = ld_row(kc.sdp + 6 * n, pos);
    k.Cg = ld_row(kc.sdp + 7 * n, pos);
    k.Cov = ld_row(kc.sdp + 8 * n, pos);
    k.Aj = J ? ld_row(kc.sdp + 9 * n, pos) : 0.0;
    return k;
}

// Evaluate the device at position pos; the card is chosen per polarity with a
// wave-uniform index (one pass per polarity present in the wave).
template <bool J = true>
__device__ __forceinline__ DevOut eval_pos(const KCirc &kc, const KCall &call, int pos,
                                           const DevIn &d, double *qout = nullptr) {
    const int isP = kc.pol[pos] < 0 ? 1 : 0;
    const DevConstT<double> k = load_consts<J>(kc, pos);
    const double Vd = volt(call.x, d.t0), Vg = volt(call.x, d.t1);
    const double Vs = volt(call.x, d.t2), Vb = volt(call.x, d.t3);
    const double *hist = call.hist ? call.hist + 4 * (size_t)kc.perm[pos] : nullptr;
    DevOut o;
    for (;;) {
        const int p0 = __builtin_amdgcn_readfirstlane(isP);
        if (isP == p0) {
            const DevCard &cd = kc.card[p0];
            const double p = p0 ? -1.0 : 1.0;
            o = eval_model<double, J>(cd, p, k, Vd, Vg, Vs, Vb, call.ag0, hist, qout);
            break;
        }
    }
    return o;
}

template <bool COHERENT>
__device__ __forceinline__ void stamp_colour(const KCirc &kc, const KCall &call, int pos,
                                             const DevIn &d, const DevOut &o) {
    double Y[16];
    full_Y(o, Y);
    const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
    ColourSinkT<COHERENT> sink{kc.code, kc.n, pos, call.A, call.b, kc.stage};
    emit_merged(d.key, Y, bl, sink);
}

template <int K, class Sink>
__device__ __forceinline__ void stamp_k(Sink &sink, const double *buf, int n, int pos) {
    double m[K * K + K];
#pragma unroll
    for (int j = 0; j < K * K + K; ++j) m[j] = buf[(size_t)j * n + pos];
    sink.template stamp<K * K, K>(m);
}
template <class Sink>
__device__ __forceinline__ void stamp_from_buffer(Sink &sink, const double *buf, int n, int pos, int k) {
    for (;;) {
        const int k0 = __builtin_amdgcn_readfirstlane(k);
        if (k == k0) {
            switch (k0) {
                case 1: stamp_k<1>(sink, buf, n, pos); break;
                case 2: stamp_k<2>(sink, buf, n, pos); break;
                case 3: stamp_k<3>(sink, buf, n, pos); break;
                case 4: stamp_k<4>(sink, buf, n, pos); break;
                default: break;
            }
            break;
        }
    }
}

// Coloured stamping of one device from its merged values in LDS rows (value of code
// row j at rows[j * stride + lane]): every load of a load-add entry is issued first
// (coherent across the XCDs), then every store; first writers store -0.0 + value.
__device__ __forceinline__ void apply_rows(const KCall &call, double *stage, const uint32_t cdv_in[NCODE], int k,
                                           const double *rows, int lane, int stride) {
    // addresses are formed here, not hoisted out of the caller's colour loop (that
    // would keep forty addresses live across the phases)
    uint32_t cdv[NCODE];
#pragma unroll
    for (int j = 0; j < NCODE; ++j) {
        cdv[j] = cdv_in[j];
        asm volatile("" : "+v"(cdv[j]));
    }
    double old[NCODE];
#pragma unroll
    for (int j = 0; j < NCODE; ++j) {
        old[j] = -0.0;
        const uint32_t tag = cdv[j] >> 30, idx = cdv[j] & 0x3FFFFFFFu;
        if (tag == TAG_ADD)
            old[j] = __hip_atomic_load((j >= k * k ? call.b : call.A) + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int j = 0; j < NCODE; ++j) {
        const uint32_t tag = cdv[j] >> 30, idx = cdv[j] & 0x3FFFFFFFu;
        if (tag == 3u) continue;
        double *p = tag == TAG_HUB ? stage + idx : (j >= k * k ? call.b : call.A) + idx;
        __hip_atomic_store(p, old[j] + rows[j * stride + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Voltage-source stamps and entries no device writes (grid-stride).
__device__ __forceinline__ void fixed_stores(const KCirc &kc, const KCall &call, int tid,
                                             int nthreads) {
    for (int i = tid; i < kc.n_fixA; i += nthreads) call.A[kc.fixA_idx[i]] = kc.fixA_val[i];
    for (int i = tid; i < kc.n_fixB; i += nthreads) call.b[kc.fixB_idx[i]] = kc.fixB_val[i];
}

__device__ __forceinline__ double ld_coherent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// s + v[i0] + v[i0+1] + ... + v[n-1], left to right, by one thread; the LDS reads
// go out sixteen at a time, the next sixteen before the current sixteen are added,
// so that their latency hides behind the dependent adds.
__device__ __forceinline__ double fold_more(double s, const double *v, int i0, int n) {
    int i = i0;
    if (i + 16 <= n) {
        double t[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) t[k] = v[i + k];
        for (i += 16; i + 16 <= n; i += 16) {
            double u[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) u[k] = v[i + k];
#pragma unroll
            for (int k = 0; k < 16; ++k) s = s + t[k];
#pragma unroll
            for (int k = 0; k < 16; ++k) t[k] = u[k];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) s = s + t[k];
    }
    for (; i < n; ++i) s = s + v[i];
    return s;
}

// Left fold of n >= 1 values in LDS by one thread.
__device__ __forceinline__ double fold_lds(const double *v, int n) { return fold_more(v[0], v, 1, n); }

__device__ __forceinline__ void hub_store(const KCirc &kc, const KCall &call, int h, double s) {
    const uint32_t tgt = (uint32_t)kc.hub_target[h];
    if (tgt & HUB_B_FLAG) call.b[tgt & ~HUB_B_FLAG] = s;
    else call.A[tgt] = s;
}

// A hub chunk's sum is known (wave-uniform call): store it if the hub has one
// chunk, else record it as a partial and count it; true when this wave recorded the
// hub's last partial (the hub's final sum is then due).
__device__ __forceinline__ bool hub_chunk_publish(const KCirc &kc, const KCall &call, int q, double s) {
    const int lane = threadIdx.x & 63;
    const int h = kc.hub_of_chunk[q];
    const int nchunk = kc.hub_cptr[h + 1] - kc.hub_cptr[h];
    if (nchunk == 1) {
        if (lane == 0) hub_store(kc, call, h, s);
        return false;
    }
    int last = 0;
    if (lane == 0) {
        st_coherent(kc.hub_part + q, s);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        last = __hip_atomic_fetch_add(kc.hub_count + (size_t)h * CNT_STRIDE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
               (uint32_t)nchunk;
    }
    return __shfl(last, 0, 64) != 0;
}

// Fixed-shape hub sum: the pairwise tree over the contributions in ascending device
// index, padded with -0.0 (the exact identity of IEEE addition) to a power of two.
// Every aligned block of HUB_K contributions is a subtree, so a hub is summed chunk
// by chunk (one wave per chunk), then the chunk sums by the same tree.

// Tree sum of cnt <= HUB_K staged values by one wave (all lanes call it, cnt
// wave-uniform): lane l adds values 4l .. 4l+3 as (v0 + v1) + (v2 + v3), then a
// butterfly adds aligned groups of 2, 4, .., 64 lanes.  IEEE addition is
// commutative bit for bit, so both lanes of a pair form the same sum and every lane
// ends with the tree's result.
static_assert(HUB_K == 4 * 64, "a hub chunk is four values per lane of one wave");
__device__ __forceinline__ double wave_tree_chunk(const double *src, int cnt) {
    const int lane = threadIdx.x & 63;
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = 4 * lane + k < cnt ? ld_coherent(src + 4 * lane + k) : -0.0;
    double s = (v[0] + v[1]) + (v[2] + v[3]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) s = s + __shfl_xor(s, off, 64);
    return s;
}

// Tree sum of a hub's cnt <= HUB_MAX_PARTS part sums by one wave (cnt wave-uniform):
// aligned groups of 256 as in wave_tree_chunk (four groups' loads issued at once),
// lane g keeping group g's sum, then a butterfly over the group sums.
static_assert(HUB_MAX_PARTS <= 64 * 256, "part sums form at most 64 groups");
__device__ __forceinline__ double wave_tree(const double *src, int cnt) {
    const int lane = threadIdx.x & 63;
    const int ng = (cnt + 255) / 256;
    double mine = -0.0;
    for (int g0 = 0; g0 < ng; g0 += 4) {
        double gs[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int e = (g0 + i) * 256 + 4 * lane + k;
                v[k] = e < cnt ? ld_coherent(src + e) : -0.0;
            }
            gs[i] = (v[0] + v[1]) + (v[2] + v[3]);
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int i = 0; i < 4; ++i) gs[i] = gs[i] + __shfl_xor(gs[i], off, 64);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (lane == g0 + i) mine = gs[i];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) mine = mine + __shfl_xor(mine, off, 64);
    return mine;
}

// The last chunk of hub h has been recorded by this wave: sum the chunk sums, store,
// and return the hub's counter to zero for the next call.
__device__ __forceinline__ void hub_finish(const KCirc &kc, const KCall &call, int h) {
    const int c0 = kc.hub_cptr[h];
    const double s = wave_tree(kc.hub_part + c0, kc.hub_cptr[h + 1] - c0);
    if ((threadIdx.x & 63) == 0) {
        hub_store(kc, call, h, s);
        __hip_atomic_store(kc.hub_count + (size_t)h * CNT_STRIDE, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Hub chunks q0 .. q1-1, one per wave (waves wave0, wave0 + nwaves, ..); the wave
// that records a hub's last chunk sum (a coherent counter) forms the hub's sum, so no
// grid barrier is needed.  Needs no workgroup barrier: each wave works alone.
__device__ __forceinline__ void hub_chunks(const KCirc &kc, const KCall &call, int q0, int q1, int wave0,
                                           int nwaves) {
    const int wave = threadIdx.x >> 6;
    for (int q = q0 + wave0 + wave; q < q1; q += nwaves) {
        const int h = kc.hub_of_chunk[q];
        const int j = q - kc.hub_cptr[h];
        const int beg = kc.hub_ptr[h] + j * HUB_K;
        const double s = wave_tree_chunk(kc.stage + beg, min(HUB_K, kc.hub_ptr[h + 1] - beg));
        if (hub_chunk_publish(kc, call, q, s)) hub_finish(kc, call, h);
    }
}

// ---- grid barrier -----------------------------------------------------------------
// Every access to data shared between colour phases (A, b, hub staging) is an
// agent-scope coherent access, so the barrier only has to order them: each wave
// waits for its outstanding memory operations (s_waitcnt 0) before the workgroup
// barrier, block i > 0 then publishes its arrival epoch in its own word, block 0
// polls all arrival words in parallel and releases everyone through one word.
// Every wait is bounded by spin_limit; on expiry the error word is set and all
// later waits fall through, so the grid always drains.
__device__ __forceinline__ uint32_t ld_flag(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void drain_memory() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ void grid_barrier(const KSync &ks, uint32_t epoch, uint32_t nblocks) {
    uint32_t *rel = ks.sync;
    uint32_t *err = ks.sync + 1;
    uint32_t *arr = ks.sync + 2;
    drain_memory();
    __syncthreads();
    if (blockIdx.x == 0) {
        for (uint32_t i = threadIdx.x + 1; i < nblocks; i += blockDim.x) {
            int64_t spins = 0;
            while (ld_flag(arr + i) != epoch) {
                __builtin_amdgcn_s_sleep(1);
                if ((++spins & 63) == 0 && (spins > ks.spin_limit || ld_flag(err) != 0)) {
                    st_flag(err, 1u);
                    break;
                }
            }
        }
        drain_memory();
        __syncthreads();
        if (threadIdx.x == 0) st_flag(rel, epoch);
    } else if (threadIdx.x == 0) {
        st_flag(arr + blockIdx.x, epoch);
        int64_t spins = 0;
        while (ld_flag(rel) != epoch) {
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 63) == 0 && (spins > ks.spin_limit || ld_flag(err) != 0)) {
                st_flag(err, 1u);
                break;
            }
        }
    }
    drain_memory();
    __syncthreads();
}

// ---- kernels ----------------------------------------------------------------------

__global__ void k_gather_params(int32_t n, const int32_t *perm, const double *W, const double *L,
                                const double *V, double *par) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int32_t v = perm[p];
        par[p] = W[v];
        par[(size_t)n + p] = L[v];
        par[2 * (size_t)n + p] = V[v];
    }
}

// One colour per launch (the per-colour parallel-for schedule).
template <bool J>
__global__ void __launch_bounds__(256) k_colour_phase(KCirc kc, KCall call, int32_t c,
                                                      int32_t with_fixed) {
    const int beg = kc.cptr[c], end = kc.cptr[c + 1];
    for (int pos = beg + blockIdx.x * blockDim.x + threadIdx.x; pos < end;
         pos += gridDim.x * blockDim.x) {
        const DevIn d = load_terms(kc, pos);
        const DevOut o = eval_pos<J>(kc, call, pos, d);
        stamp_colour<false>(kc, call, pos, d, o);
    }
    if (with_fixed) fixed_stores(kc, call, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_fixed(KCirc kc, KCall call) {
    fixed_stores(kc, call, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Linear part (series resistors) of entries that devices also write, after the
// device contributions: one entry per lane, each listed once.
__global__ void __launch_bounds__(256) k_linear_add(int32_t n, const int32_t *__restrict__ idx,
                                                     const double *__restrict__ val, double *__restrict__ A) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int32_t s = idx[i];
        A[s] = A[s] + val[i];
    }
}

// Newton update after the solve (y = solution of A y = b at the present x).  The
// clamp compares explicitly so that a NaN step stays NaN; the largest |d| of the
// block is reduced in LDS and merged with one 64-bit atomic max on its bits (the
// order of non-negative doubles, NaN above infinity).
__global__ void __launch_bounds__(256) k_newton_update(int32_t n, int32_t n_clamp,
                                                       const uint8_t *__restrict__ clamp,
                                                       const double *__restrict__ y, double *__restrict__ x,
                                                       double vstep, unsigned long long *step_bits) {
    __shared__ unsigned long long red[256];
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long m = 0;
    if (i < n) {
        double d = y[i] - x[i];
        if (clamp ? clamp[i] != 0 : i < n_clamp) {
            if (d > vstep) d = vstep;
            else if (d < -vstep) d = -vstep;
        }
        x[i] = x[i] + d;
        m = (unsigned long long)__double_as_longlong(fabs(d));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(step_bits, red[0]);
}

__global__ void __launch_bounds__(256) k_hub(KCirc kc, KCall call) {
    hub_chunks(kc, call, 0, kc.n_hub_chunks, blockIdx.x * (blockDim.x >> 6), gridDim.x * (blockDim.x >> 6));
}

// Circuits stamped inside one workgroup (batches): colour phases separated by
// workgroup barriers, each device evaluated in its phase, then the circuit's own
// hub chunks.
template <bool J>
__device__ __forceinline__ void local_circuits(const KCirc &kc, const KCall &call, const KLocal &kl, int first,
                               int stride) {
    for (int li = first; li < kl.n; li += stride) {
        const int32_t *t = kl.table + 6 * (size_t)li;
        const int32_t cp = t[2], nc = t[3];
        for (int c = 0; c < nc; ++c) {
            const int beg = kl.cptr[cp + c], end = kl.cptr[cp + c + 1];
            for (int pos = beg + (int)threadIdx.x; pos < end; pos += blockDim.x) {
                const DevIn d = load_terms(kc, pos);
                const DevOut o = eval_pos<J>(kc, call, pos, d);
                stamp_colour<true>(kc, call, pos, d, o);
            }
            drain_memory();
            __syncthreads();
        }
        hub_chunks(kc, call, t[4], t[5], 0, blockDim.x >> 6);
    }
}

// Persistent coloured kernel.  Blocks [0, n_part) run the colour schedule with
// grid barriers among themselves over positions [0, cptr[n_colors]); blocks from
// n_part on stamp the workgroup-local circuits.  MODE 0: evaluate inside each colour
// phase (grid-stride).  MODE 1: every thread evaluates its own device before the
// first phase and keeps the merged values in LDS (requires n_part*block >= the
// scheduled positions; dynamic LDS of nc_max doubles per thread).  MODE 2: stamp
// phases only, merged values read from the buffer of k_eval_buffer.
template <int MODE, bool LOCAL, bool J>
__device__ __forceinline__ void persistent_body(const KCirc &kc, const KCall &call,
                                                const KSync &ks, const double *buf, int n_part,
                                                int n_global_chunks, const KLocal &kl) {
    __shared__ uint32_t base_s;
    if (blockIdx.x == 0) fixed_stores(kc, call, threadIdx.x, blockDim.x);
    if constexpr (LOCAL) {
        if ((int)blockIdx.x >= n_part) {
            local_circuits<J>(kc, call, kl, blockIdx.x - n_part, gridDim.x - n_part);
            return;
        }
    }
    if (threadIdx.x == 0) base_s = ld_flag(ks.sync);
    __syncthreads();
    const uint32_t base = base_s;
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthr = n_part * blockDim.x;

    const int n_sched = kc.cptr[kc.n_colors];
    // MODE 1: every thread evaluates and merges its own device first; the merged values
    // wait in LDS ([code row][thread]), the code words in registers (tag 3 = unused)
    extern __shared__ double rows[];
    uint32_t cdv[NCODE];
    int kq = 0;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int j = 0; j < NCODE; ++j) cdv[j] = 0xC0000000u;
        if (gtid < n_sched) {
            const DevIn d = load_terms(kc, gtid);
            const DevOut o = eval_pos<J>(kc, call, gtid, d);
            double Y[16];
            full_Y(o, Y);
            const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
            LdsRowSink sink{rows + threadIdx.x, (int)blockDim.x};
            emit_merged(d.key, Y, bl, sink);
            kq = (d.t0 != 0) + (d.t1 != 0 && d.t1 != d.t0) + (d.t2 != 0 && d.t2 != d.t0 && d.t2 != d.t1) +
                 (d.t3 != 0 && d.t3 != d.t0 && d.t3 != d.t1 && d.t3 != d.t2);
#pragma unroll
            for (int j = 0; j < NCODE; ++j)
                if (j < kq * kq + kq) cdv[j] = (uint32_t)kc.code[(size_t)j * kc.n + gtid];
        }
    }
    uint32_t epoch = base;
    for (int c = 0; c < kc.n_colors; ++c) {
        const int beg = kc.cptr[c], end = kc.cptr[c + 1];
        if constexpr (MODE == 1) {
            if (gtid >= beg && gtid < end) apply_rows(call, kc.stage, cdv, kq, rows, threadIdx.x, blockDim.x);
        } else {
            for (int pos = beg + gtid; pos < end; pos += nthr) {
                const DevIn dd = load_terms(kc, pos);
                if constexpr (MODE == 0) {
                    const DevOut oo = eval_pos<J>(kc, call, pos, dd);
                    stamp_colour<true>(kc, call, pos, dd, oo);
                } else {
                    const int k = (dd.t0 != 0) + (dd.t1 != 0 && dd.t1 != dd.t0) +
                                  (dd.t2 != 0 && dd.t2 != dd.t0 && dd.t2 != dd.t1) +
                                  (dd.t3 != 0 && dd.t3 != dd.t0 && dd.t3 != dd.t1 && dd.t3 != dd.t2);
                    ColourSinkT<true> sink{kc.code, kc.n, pos, call.A, call.b, kc.stage};
                    stamp_from_buffer(sink, buf, kc.n, pos, k);
                }
            }
        }
        if (c + 1 < kc.n_colors || n_global_chunks > 0) grid_barrier(ks, ++epoch, n_part);
    }
    hub_chunks(kc, call, 0, n_global_chunks, blockIdx.x * (blockDim.x >> 6), n_part * (blockDim.x >> 6));
}

template <bool J>
__global__ void __launch_bounds__(256) k_persistent_phase(KCirc kc, KCall call, KSync ks,
                                                          const double *buf, int n_part,
                                                          int n_global_chunks, KLocal kl) {
    persistent_body<0, true, J>(kc, call, ks, buf, n_part, n_global_chunks, kl);
}
// Evaluate-ahead keeps one device's merged values per thread across the colour
// phases (in LDS); it needs every device resident at once, hence four waves per SIMD.
template <bool J>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_persistent_ahead(KCirc kc, KCall call, KSync ks, const double *buf, int n_part,
                   int n_global_chunks, KLocal kl) {
    persistent_body<1, true, J>(kc, call, ks, buf, n_part, n_global_chunks, kl);
}
// The same without workgroup-local circuits (single circuits): less register
// pressure in the one path it has.
template <bool J>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_persistent_ahead_single(KCirc kc, KCall call, KSync ks, const double *buf, int n_part,
                          int n_global_chunks, KLocal kl) {
    persistent_body<1, false, J>(kc, call, ks, buf, n_part, n_global_chunks, kl);
}
template <bool J>
__global__ void __launch_bounds__(256) k_persistent_stamp(KCirc kc, KCall call, KSync ks,
                                                          const double *buf, int n_part,
                                                          int n_global_chunks, KLocal kl) {
    persistent_body<2, true, J>(kc, call, ks, buf, n_part, n_global_chunks, kl);
}

// History terms of the next backward-Euler step: ag0 times each device's terminal
// charges at x, written in original device order (4 per device: d, g, s, b).
__global__ void __launch_bounds__(256) k_history(KCirc kc, KCall call, double *hist_out) {
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < kc.n; pos += gridDim.x * blockDim.x) {
        const DevIn d = load_terms(kc, pos);
        double q[4];
        (void)eval_pos(kc, call, pos, d, q);
        double *h = hist_out + 4 * (size_t)kc.perm[pos];
        h[0] = call.ag0 * q[0];
        h[1] = call.ag0 * q[1];
        h[2] = call.ag0 * q[2];
        h[3] = call.ag0 * q[3];
    }
}

hipError_t launch_history(const KCirc &kc, const KCall &call, double *hist_out, hipStream_t s) {
    if (kc.n == 0) return hipSuccess;
    const int grid = std::max(1, std::min(4096, (kc.n + 255) / 256));
    hipLaunchKernelGGL(k_history, dim3(grid), dim3(256), 0, s, kc, call, hist_out);
    return hipGetLastError();
}

// Evaluate every device and write its merged values (buffered variant).
template <bool J>
__global__ void __launch_bounds__(256) k_eval_buffer(KCirc kc, KCall call, double *buf) {
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < kc.n; pos += gridDim.x * blockDim.x) {
        const DevIn d = load_terms(kc, pos);
        const DevOut o = eval_pos<J>(kc, call, pos, d);
        double Y[16];
        full_Y(o, Y);
        const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
        BufferSink sink{buf, kc.n, pos};
        emit_merged(d.key, Y, bl, sink);
    }
}

// Serial stamping after the buffered evaluation (the paper's loadomp form): one lane
// adds every device's merged values, devices in ascending index, onto the zeroed A
// and b, i.e. the serial order of accumulation.  The fixed stores touch other
// entries and are made by the whole wave first.
__global__ void __launch_bounds__(64) k_serial_stamp(KCirc kc, KCall call, const double *buf,
                                                     const int32_t *ipos) {
    fixed_stores(kc, call, threadIdx.x, blockDim.x);
    if (threadIdx.x != 0) return;
    for (int32_t v = 0; v < kc.n; ++v) {
        const int32_t p = ipos[v];
        const DevIn d = load_terms(kc, p);
        const int k = (d.t0 != 0) + (d.t1 != 0 && d.t1 != d.t0) + (d.t2 != 0 && d.t2 != d.t0 && d.t2 != d.t1) +
                      (d.t3 != 0 && d.t3 != d.t0 && d.t3 != d.t1 && d.t3 != d.t2);
        for (int j = 0; j < k * k + k; ++j) {
            double *dst = (j < k * k ? call.A : call.b) + kc.acode[(size_t)j * kc.n + p];
            *dst = *dst + buf[(size_t)j * kc.n + p];
        }
    }
}

__global__ void k_fill_zero(double *A, int64_t nA, double *b, int64_t nb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nA + nb;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < nA) A[i] = 0.0; else b[i - nA] = 0.0;
    }
}

// Atomic variant: no colouring; every contribution is an FP64 atomic add.
template <bool J>
__global__ void __launch_bounds__(256) k_atomic(KCirc kc, KCall call) {
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x, nthr = gridDim.x * blockDim.x;
    for (int pos = gtid; pos < kc.n; pos += nthr) {
        const DevIn d = load_terms(kc, pos);
        const DevOut o = eval_pos<J>(kc, call, pos, d);
        double Y[16];
        full_Y(o, Y);
        const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
        AtomicSink sink{kc.acode, kc.n, pos, call.A, call.b};
        emit_merged(d.key, Y, bl, sink);
    }
    fixed_stores(kc, call, gtid, nthr);
}

// Atomic variant with wave-level pre-reduction of the hub (rail) entries: every
// other contribution is an FP64 atomic add as in k_atomic; a wave's contributions to
// one hub target are summed over the wave (a butterfly) and added by one lane.
template <bool J>
__global__ void __launch_bounds__(256) k_atomic_wave(KCirc kc, KCall call) {
    constexpr int HS = 4;
    const int lane = threadIdx.x & 63;
    const int nthr = gridDim.x * blockDim.x;
    // wave-uniform trip count: every lane of a wave takes part in the reductions
    for (int base = blockIdx.x * blockDim.x + ((int)threadIdx.x & ~63); base < kc.n; base += nthr) {
        const int pos = base + lane;
        AtomicHubSink<HS> sink{kc.acode, kc.code, kc.n, pos, call.A, call.b};
        if (pos < kc.n) {
            const DevIn d = load_terms(kc, pos);
            const DevOut o = eval_pos<J>(kc, call, pos, d);
            double Y[16];
            full_Y(o, Y);
            const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
            emit_merged(d.key, Y, bl, sink);
        }
#pragma unroll
        for (int s = 0; s < HS; ++s) {
            int32_t t = s < sink.nh ? sink.tgt[s] : -1;
            const double v = s < sink.nh ? sink.val[s] : -0.0;
            uint64_t act = __ballot(t != -1);
            while (act) {
                const int leader = __builtin_ctzll(act);
                const int32_t t0 = __shfl(t, leader, 64);
                double x = t == t0 ? v : -0.0;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) x = x + __shfl_xor(x, off, 64);
                if (lane == leader) {
                    const uint32_t u = (uint32_t)t0;
                    (void)unsafeAtomicAdd((u & HUB_B_FLAG ? call.b : call.A) + (u & ~HUB_B_FLAG), x);
                }
                if (t == t0) t = -1;
                act = __ballot(t != -1);
            }
        }
    }
    fixed_stores(kc, call, blockIdx.x * blockDim.x + threadIdx.x, nthr);
}

// ---- region schedule ------------------------------------------------------------
// One workgroup per region.  The region's devices are evaluated at once (NMOS lanes
// first, then PMOS lanes) and their merged values parked in LDS rows.  An entry
// written by one or two devices of the region accumulates in an LDS slot by LDS
// atomic adds (exact in any order for two writers); an entry written by more devices
// of the region is folded by one lane from the parked values in colour order; a hub
// part whose contributions all come from the region is summed from LDS.
// Contributions to entries shared with other regions and to hub parts spanning
// regions are staged in global memory, and each such entry or part is folded by the
// last region that contributes to it (an arrival counter, counted right after the
// LDS adds so that its round trip overlaps the lane folds).  Follow-up kernels fold
// the large shared entries and sum each hub's parts.  No wave ever waits for another
// workgroup.

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// (lgkmcnt 0), not for its global stores, which a full __syncthreads would drain.
// The signal fences keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ void store_target(const KCall &call, uint32_t tgt, double s) {
    const uint32_t idx = tgt & 0x3FFFFFFFu;
    if ((tgt >> 30) == ITEM_B) call.b[idx] = s;
    else call.A[idx] = s;
}

// Fold of the items this thread's region was the last to reach (last: that region;
// shared entries one lane each, in colour order; hub parts spanning regions one wave
// each, by the tree, stored as parts).  Called by every lane of the wave.
__device__ __forceinline__ void fold_item(const KCirc &kc, const KCall &call, bool last, int beg, int cnt,
                                          uint32_t tgt) {
    const int lane = threadIdx.x & 63;
    const bool hub = (tgt >> 30) == ITEM_HUB;
    if (last && !hub) {   // shared entry, at most ITEM_LANE_MAX contributions
        double v[ITEM_LANE_MAX];
#pragma unroll
        for (int k = 0; k < ITEM_LANE_MAX; ++k) v[k] = k < cnt ? ld_coherent(kc.stage + beg + k) : 0.0;
        double sum = v[0];
#pragma unroll
        for (int k = 1; k < ITEM_LANE_MAX; ++k)
            if (k < cnt) sum = sum + v[k];
        store_target(call, tgt, sum);
    }
    uint64_t big = __ballot(last && hub);
    while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int bbeg = __shfl(beg, l, 64), bcnt = __shfl(cnt, l, 64);
        const int q = (int)((uint32_t)__shfl((int)tgt, l, 64) & 0x3FFFFFFFu);
        const double sum = wave_tree_chunk(kc.stage + bbeg, bcnt);
        if (lane == 0) kc.hub_part[q] = sum;
    }
}

// An item's arrival counter after the last of its regions has counted: back to 0 for
// the next call.
__device__ __forceinline__ void reset_count(const KRegion &kr, int it) {
    __hip_atomic_store(kr.item_count + (size_t)it * CNT_STRIDE, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Items of one region in [jb, je) of its links, after its staged values are complete:
// count the arrival; the last region of an item folds it (fold_item; consecutive
// items go to different waves).  Called by every thread of the workgroup.  The hub
// sums over the parts follow in the follow-up kernel (k_region_tail).
__device__ __forceinline__ void finish_items(const KCirc &kc, const KCall &call, const KRegion &kr, int jb, int je,
                                             bool hub_only = false) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int base = jb; base < je; base += blockDim.x) {
        const int i = base + lane * nw + wave;
        int beg = 0, cnt = 0;
        uint32_t tgt = 0;
        bool last = false;
        if (i < je && !(hub_only && ((uint32_t)kr.item[4 * (size_t)kr.ritems[i] + 2] >> 30) != ITEM_HUB)) {
            const int it = kr.ritems[i];
            const int32_t *f = kr.item + 4 * (size_t)it;
            beg = f[0];
            cnt = f[1];
            tgt = (uint32_t)f[2];
            const int need = f[3];
            if (need == 1) {
                last = true;
            } else {
                last = __hip_atomic_fetch_add(kr.item_count + (size_t)it * CNT_STRIDE, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) + 1 == (uint32_t)need;
                if (last) reset_count(kr, it);
            }
        }
        fold_item(kc, call, last, beg, cnt, tgt);
    }
}

// Tree sum of 16 values.
__device__ __forceinline__ double tree16(const double *v) {
    return (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) +
           (((v[8] + v[9]) + (v[10] + v[11])) + ((v[12] + v[13]) + (v[14] + v[15])));
}

// Follow-up of the region schedule, one workgroup of 256 threads: hub h summed from
// its parts (complete at kernel start) by the pairwise tree.  Its P parts, padded
// with -0.0 to 256 * S (S parts per lane, a power of two), are cut into one aligned
// stripe of S per lane, each a subtree: a lane sums its stripe in up to four blocks
// of 16 (every load issued before the sums), a butterfly sums the stripes of a wave,
// thread 0 the four wave sums.
static_assert(HUB_MAX_PARTS <= 256 * 4 * 16, "a hub's parts fit four blocks of 16 per lane");
__device__ __forceinline__ void hub_parts_block(const KCirc &kc, const KCall &call, int h) {
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = kc.hub_cptr[h], P = kc.hub_cptr[h + 1] - c0;
    const double *src = kc.hub_part + c0;
    int S = 1;
    while (S * 256 < P) S <<= 1;
    const int base = (int)threadIdx.x * S;
    const int nb = S >= 16 ? S / 16 : 1;
    double bs[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int e = base + b * 16 + k;
            v[k] = (b < nb && k < S && e < P) ? src[e] : -0.0;
        }
        bs[b] = tree16(v);
    }
    double acc = (bs[0] + bs[1]) + (bs[2] + bs[3]);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc = acc + __shfl_xor(acc, off, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) hub_store(kc, call, h, (red[0] + red[1]) + (red[2] + red[3]));
}

// Region schedule body.  GRID = false: the region kernel (shared entries staged and
// folded by the last contributing region).  GRID = true: the same inside one
// persistent launch (every region resident, one workgroup each): shared entries are
// written in place, level by level in colour order (first writer stores, later ones
// load-add, coherent across XCDs), with a grid-wide barrier between levels; then the
// hub sums.
template <bool GRID, bool J>
__device__ __forceinline__ void region_body(const KCirc &kc, const KCall &call, const KRegion &kr, const KSync &ks) {
    // LDS: kr.lds_int accumulators, then kr.nc_max merged values per lane
    extern __shared__ double lds[];
    __shared__ uint32_t base_s;
    fixed_stores(kc, call, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
    if constexpr (GRID) {
        if (threadIdx.x == 0) base_s = ld_flag(ks.sync);
    } else {
        if ((int)blockIdx.x >= kr.n_regions) return;
    }
    // (the grid form is launched with exactly one workgroup per region; a workgroup
    // beyond them would own nothing and only take part in the barriers)
    int f[RT_FIELDS] = {};
    if ((int)blockIdx.x < kr.n_regions) {
        const int32_t *rt = kr.rtab + (size_t)blockIdx.x * RT_FIELDS;
#pragma unroll
        for (int k = 0; k < RT_FIELDS; ++k) f[k] = rt[k];
    }
    const int p0 = f[0], nN = f[1], nP = f[2], ib = f[4], ie = f[5], jb = f[6], je = f[7];
    const int fb = f[8], fe = f[9], hb = f[10], he = f[11];
    const int t = threadIdx.x;
    const int pos = t < nN + nP ? p0 + t : -1;
    // the region's accumulators start at -0.0, the exact identity of IEEE addition, so
    // a first writer's load-add equals its store (visible after the barrier below)
    for (int i = t; i < (ie - ib) + RHUB_K * (he - hb); i += blockDim.x) lds[i] = -0.0;
    // part index of this lane's first local hub part, loaded now (used after the LDS adds)
    int hq0 = 0;
    {
        const int i0 = hb + (t >> 6) * 8 + ((t & 63) >> 3);
        if (i0 < he) hq0 = kr.hfold[i0];
    }
    // evaluate and merge at once (all waves in parallel); the merged values go to LDS
    // rows [code row][lane], where the lane folds read them, and in the region form
    // also stay in registers for the staging stores and the LDS adds
    double *mst = lds + kr.lds_int;
    const int B = blockDim.x;
    // code words, loaded right after the evaluation (the loads overlap the merge) on
    // the lanes holding a device.  Only rows j < ncm are read (ncm, the largest row
    // count of any device, is the same on every lane; the rows of a device beyond its
    // own count hold tag 3, unused); the loads of the rows beyond ncm repeat row
    // ncm - 1, so that every load is unconditional.
    const int ncm = kr.nc_max;
    uint32_t cd[NCODE];
    double mv[NCODE];   // the merged values, also kept in registers for the region form
    if (pos >= 0) {
        const DevIn d = load_terms(kc, pos);
        const DevOut o = eval_pos<J>(kc, call, pos, d);
#pragma unroll
        for (int j = 0; j < NCODE; ++j) cd[j] = (uint32_t)ld_row(kc.code + (size_t)min(j, ncm - 1) * kc.n, pos);
        double Y[16];
        full_Y(o, Y);
        const double bl[4] = {o.bd, o.bg, o.bs, o.bb};
        if constexpr (GRID) {
            LdsRowSink sink{mst + t, B};
            emit_merged(d.key, Y, bl, sink);
        } else {
            LdsRowRegSink sink{mst + t, B, mv};
            emit_merged(d.key, Y, bl, sink);
        }
    }
    // tables the tail needs, loaded now (their latency overlaps the staging and the LDS
    // adds): this lane's lane fold and its first sources, its first item, its
    // owned-entry targets
    constexpr int OWN_PF = 4;
    const int fi = fb + t;
    int fd_t = 0, fd_s = 0, fd_c = 0;
    int32_t fsrc[FOLD_HEAD] = {};
    if (fi < fe) {
        const int32_t *fd = kr.fold + 3 * (size_t)fi;
        fd_t = fd[0];
        fd_s = fd[1];
        fd_c = fd[2];
        static_assert(FOLD_HEAD == 4, "one 16-byte load per fold head");
        const int4 h = *reinterpret_cast<const int4 *>(kr.fold_head + FOLD_HEAD * (size_t)fi);
        fsrc[0] = h.x;
        fsrc[1] = h.y;
        fsrc[2] = h.z;
        fsrc[3] = h.w;
    }
    const int nw0 = blockDim.x >> 6;
    const int ii0 = jb + (t & 63) * nw0 + (t >> 6);
    int4 ih = make_int4(0, 0, 0, 0);   // this thread's item of the first round (KRegion::ritem_head)
    if (!GRID && ii0 < je) ih = *reinterpret_cast<const int4 *>(kr.ritem_head + 4 * (size_t)ii0);
    uint32_t own_t[OWN_PF];
#pragma unroll
    for (int k = 0; k < OWN_PF; ++k) own_t[k] = t + k * B < ie - ib ? (uint32_t)kr.int_target[ib + t + k * B] : 0u;
    // values of shared entries and hubs: staged at once (no order among them); the grid
    // form stages only the hub values
    if (pos >= 0) {
#pragma unroll
        for (int j = 0; j < NCODE; ++j) {
            if (j >= ncm || (cd[j] >> 30) != TAG_STAGE) continue;
            const uint32_t sl = cd[j] & 0x3FFFFFFFu;
            if (GRID && kr.slot_first[sl] < SLOT_HUB) continue;
            st_coherent(kc.stage + sl, GRID ? mst[j * B + t] : mv[j]);
        }
    }
    lds_barrier();
    // entries of the region with one or two writers: every device adds its merged
    // values to their LDS slots with LDS atomic adds, all devices at once (the slots
    // start at -0.0, the identity, and two writers commute exactly: a + b = b + a, so
    // the sum is the colour order's whichever add lands first)
    if (pos >= 0) {
#pragma unroll
        for (int j = 0; j < NCODE; ++j) {
            if (j < ncm && (cd[j] >> 30) <= TAG_LDS_STORE)
                (void)__hip_atomic_fetch_add(lds + (cd[j] & 0x3FFFFFFFu), GRID ? mst[j * B + t] : mv[j],
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    // the region form counts its arrivals right after this barrier, so each wave's
    // staged values must be complete before it
    if constexpr (!GRID) drain_memory();
    lds_barrier();
    // arrivals at the items of the first round, counted now: their round trip overlaps
    // the lane folds and the local hub parts
    const int need0 = ih.w >> ITEM_NEED_SHIFT;
    uint32_t arr0 = 0;
    if (!GRID && ii0 < je && need0 > 1)
        arr0 = __hip_atomic_fetch_add(kr.item_count + (size_t)ih.x * CNT_STRIDE, 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    // lane folds: entries of the region with many writers, one lane each, the
    // writers' merged values read from LDS in colour order (no phase per writer)
    for (int i = fb + t; i < fe; i += B) {
        int tg = fd_t, sb = fd_s, cnt = fd_c;
        if (i != fi) {
            const int32_t *fd = kr.fold + 3 * (size_t)i;
            tg = fd[0];
            sb = fd[1];
            cnt = fd[2];
        }
        const int32_t *src = kr.fold_src + sb;
        double s;
        if (i == fi) {
            s = mst[(fsrc[0] >> 16) * B + (fsrc[0] & 0xFFFF)];
#pragma unroll
            for (int k = 1; k < FOLD_HEAD; ++k)
                if (k < cnt) s = s + mst[(fsrc[k] >> 16) * B + (fsrc[k] & 0xFFFF)];
            for (int k = FOLD_HEAD; k < cnt; ++k) s = s + mst[(src[k] >> 16) * B + (src[k] & 0xFFFF)];
        } else {
            s = mst[(src[0] >> 16) * B + (src[0] & 0xFFFF)];
#pragma unroll 8
            for (int k = 1; k < cnt; ++k) s = s + mst[(src[k] >> 16) * B + (src[k] & 0xFFFF)];
        }
        store_target(call, (uint32_t)tg, s);
    }
    // local hub parts: eight lanes per part, four of its LDS slots each (slots beyond
    // the part's contributions hold -0.0), a butterfly over the eight lanes: the part's
    // subtree of the hub's pairwise sum, stored as its part
    static_assert(RHUB_K == 8 * 4, "a local hub part is eight lanes of four values");
    {
        const int n_owned = ie - ib;
        int round = 0;
        for (int base = hb + (t >> 6) * 8; base < he; base += (B >> 6) * 8, ++round) {
            const int i = base + ((t & 63) >> 3);
            const int r = t & 7;
            double v[4] = {-0.0, -0.0, -0.0, -0.0};
            int q = hq0;
            if (i < he) {
                if (round > 0) q = kr.hfold[i];
                const double *src = lds + n_owned + RHUB_K * (i - hb) + 4 * r;
#pragma unroll
                for (int k = 0; k < 4; ++k) v[k] = src[k];
            }
            double sum = (v[0] + v[1]) + (v[2] + v[3]);
            sum = sum + __shfl_xor(sum, 1, 64);
            sum = sum + __shfl_xor(sum, 2, 64);
            sum = sum + __shfl_xor(sum, 4, 64);
            if (i < he && r == 0) kc.hub_part[q] = sum;
        }
    }
    if constexpr (GRID) {
        // the region's own entries, then the shared entries level by level, then the
        // hub sums by arrival counting (they need no grid barrier; their fold scratch
        // reuses the merged-value rows, so they come last)
        for (int i = t; i < ie - ib; i += blockDim.x) store_target(call, (uint32_t)kr.int_target[ib + i], lds[i]);
        const int gl = pos >= 0 ? (int)kr.glevel[pos] : -1;
        uint32_t epoch = base_s;
        for (int g = 0; g < kr.max_glevel; ++g) {
            if (gl == g) {
                // this device's shared entries: all loads, then all stores
                double old[NCODE];
#pragma unroll
                for (int j = 0; j < NCODE; ++j) {
                    old[j] = -0.0;
                    if (j >= ncm || (cd[j] >> 30) != TAG_STAGE) continue;
                    const uint32_t sl = cd[j] & 0x3FFFFFFFu;
                    if (kr.slot_first[sl] == SLOT_ADD) {
                        const uint32_t tg = (uint32_t)kr.slot_tgt[sl];
                        old[j] = ld_coherent(((tg >> 30) == ITEM_B ? call.b : call.A) + (tg & 0x3FFFFFFFu));
                    }
                }
#pragma unroll
                for (int j = 0; j < NCODE; ++j) {
                    if (j >= ncm || (cd[j] >> 30) != TAG_STAGE) continue;
                    const uint32_t sl = cd[j] & 0x3FFFFFFFu;
                    if (kr.slot_first[sl] >= SLOT_HUB) continue;
                    const uint32_t tg = (uint32_t)kr.slot_tgt[sl];
                    st_coherent(((tg >> 30) == ITEM_B ? call.b : call.A) + (tg & 0x3FFFFFFFu), old[j] + mst[j * B + t]);
                }
            }
            if (g + 1 < kr.max_glevel) grid_barrier(ks, ++epoch, gridDim.x);
        }
        drain_memory();
        __syncthreads();
        finish_items(kc, call, kr, jb, je, true);
    } else {
        // the items of the first round (arrivals counted above), then any later rounds;
        // the region's own entries are stored last (nothing waits for them).  The empty
        // asm is the first use of the counted value, so that its wait stays here and is
        // not pulled up to the atomic
        asm volatile("" : "+v"(arr0));
        const bool last0 = ii0 < je && (need0 == 1 || arr0 + 1 == (uint32_t)need0);
        if (last0 && need0 > 1) reset_count(kr, ih.x);
        fold_item(kc, call, last0, ih.y, ih.w & ((1 << ITEM_NEED_SHIFT) - 1), (uint32_t)ih.z);
        if (jb + B < je) finish_items(kc, call, kr, jb + B, je);
#pragma unroll
        for (int k = 0; k < OWN_PF; ++k)
            if (t + k * B < ie - ib) store_target(call, own_t[k], lds[t + k * B]);
        for (int i = t + OWN_PF * B; i < ie - ib; i += blockDim.x)
            store_target(call, (uint32_t)kr.int_target[ib + i], lds[i]);
    }
}

template <bool J>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_region(KCirc kc, KCall call, KRegion kr) {
    const KSync none{nullptr, 0};
    region_body<false, J>(kc, call, kr, none);
}

// Grid-barrier form: launched with one resident workgroup per region (cooperative
// launch, or an ordinary one that the occupancy query says fits at once).
template <bool J>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_region_grid(KCirc kc, KCall call, KRegion kr, KSync ks) {
    region_body<true, J>(kc, call, kr, ks);
}

// Follow-up of the region schedule, one workgroup of 256 threads: large shared
// entries i0 .. i0 + FOLD_E - 1, their staged contributions folded left in colour
// order (complete at kernel start).  In each round the workgroup loads up to FOLD_CAP
// contributions of each of its entries at once (one memory round trip for all of
// them) into one LDS row per entry, and thread e folds row e, continuing from the
// previous round for entries longer than FOLD_CAP.  The rows are padded by one value
// so that the folding threads read from different banks.
constexpr int FOLD_E = 8;
constexpr int FOLD_CAP = 512;
constexpr int FOLD_ROW = FOLD_CAP + 1;
static_assert(FOLD_CAP % 256 == 0, "a row is loaded in whole workgroups");
__device__ __forceinline__ void fold_items_block(const KCirc &kc, const KCall &call, const KRegion &kr, int i0) {
    __shared__ double rows[FOLD_E * FOLD_ROW];
    const int lane = threadIdx.x;
    // the entries of this workgroup (the same on every lane) and the folding lane's own
    int beg[FOLD_E], cnt[FOLD_E];
    int maxc = 0;
#pragma unroll
    for (int e = 0; e < FOLD_E; ++e) {
        beg[e] = 0;
        cnt[e] = 0;
        if (i0 + e < kr.n_deferred) {
            const int32_t *f = kr.item + 4 * (size_t)kr.deferred[i0 + e];
            beg[e] = f[0];
            cnt[e] = f[1];
        }
        maxc = max(maxc, cnt[e]);
    }
    int my_cnt = 0;
    uint32_t my_tgt = 0;
    if (lane < FOLD_E && i0 + lane < kr.n_deferred) {
        const int32_t *f = kr.item + 4 * (size_t)kr.deferred[i0 + lane];
        my_cnt = f[1];
        my_tgt = (uint32_t)f[2];
    }
    double s = 0.0;
    for (int p = 0; p < maxc; p += FOLD_CAP) {
        constexpr int K = FOLD_CAP / 256;
        double v[FOLD_E][K];
#pragma unroll
        for (int e = 0; e < FOLD_E; ++e)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int idx = p + k * 256 + lane;
                v[e][k] = idx < cnt[e] ? kc.stage[(size_t)beg[e] + idx] : 0.0;
            }
        if (p > 0) __syncthreads();   // the previous round's rows are folded
#pragma unroll
        for (int e = 0; e < FOLD_E; ++e)
#pragma unroll
            for (int k = 0; k < K; ++k) rows[e * FOLD_ROW + k * 256 + lane] = v[e][k];
        __syncthreads();
        const int n = min(FOLD_CAP, my_cnt - p);
        if (n > 0) s = p == 0 ? fold_lds(rows + lane * FOLD_ROW, n) : fold_more(s, rows + lane * FOLD_ROW, 0, n);
    }
    if (my_cnt > 0) store_target(call, my_tgt, s);
}

// The follow-ups of a region launch in one kernel: workgroups [0, n_fold) fold the
// large shared entries (FOLD_E each), the next n_hub sum one hub each.  The two sets
// touch different entries and read only what the region kernel completed.
__global__ void __launch_bounds__(256) k_region_tail(KCirc kc, KCall call, KRegion kr, int32_t n_fold) {
    if ((int)blockIdx.x < n_fold) fold_items_block(kc, call, kr, (int)blockIdx.x * FOLD_E);
    else hub_parts_block(kc, call, (int)blockIdx.x - n_fold);
}

__global__ void k_permute_rows(int32_t n, const int32_t *idx, const double *src, int32_t n_src, int32_t rows,
                               double *dst) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int32_t q = idx[p];
        for (int r = 0; r < rows; ++r) dst[(size_t)r * n + p] = src[(size_t)r * n_src + q];
    }
}

// Per-device constants of every position from W, L, VTH0 (kc.par) and the card of
// its polarity, written to sdp[NSD][n].
__global__ void __launch_bounds__(256) k_dev_const(KCirc kc, double *sdp) {
    const size_t n = (size_t)kc.n;
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < kc.n; pos += gridDim.x * blockDim.x) {
        const int isP = kc.pol[pos] < 0 ? 1 : 0;
        const double W = kc.par[pos], L = kc.par[n + pos], V = kc.par[2 * n + pos];
        DevConstT<double> k;
        for (;;) {
            const int p0 = __builtin_amdgcn_readfirstlane(isP);
            if (isP == p0) {
                k = dev_const(kc.card[p0], p0 ? -1.0 : 1.0, W, L, V);
                break;
            }
        }
        sdp[pos] = k.vth_s;
        sdp[n + pos] = k.dibl;
        sdp[2 * n + pos] = k.nsce;
        sdp[3 * n + pos] = k.beta0;
        sdp[4 * n + pos] = k.lambda;
        sdp[5 * n + pos] = k.k1AbL;
        sdp[6 * n + pos] = k.esatn;
        sdp[7 * n + pos] = k.Cg;
        sdp[8 * n + pos] = k.Cov;
        sdp[9 * n + pos] = k.Aj;
    }
}

// ---- host launchers ----------------------------------------------------------------

static hipError_t occupancy(const void *fn, int block, int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

// Kernels come in two instantiations: with the junction terms (J) and without them
// (cards with jmod = 0: model M's code exactly, its register allocation unchanged).
static bool junctions(const KCirc &kc) { return kc.card[0].jmod != 0.0 || kc.card[1].jmod != 0.0; }

// Resident blocks per CU that both instantiations of a kernel reach.
static hipError_t occupancy_both(const void *f0, const void *f1, int block, size_t shm, int *blocks_per_cu) {
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, f0, block, shm);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f1, block, shm);
    *blocks_per_cu = std::min(a, b);
    return e;
}

static size_t persistent_lds(int mode, int block, int nc_max) {
    return mode == 1 ? sizeof(double) * (size_t)nc_max * block : 0;
}

hipError_t persistent_capacity(int mode, int block, int nc_max, int *blocks_per_cu) {
    const void *f0 = mode == 1 ? (const void *)k_persistent_ahead<false>
                   : mode == 2 ? (const void *)k_persistent_stamp<false> : (const void *)k_persistent_phase<false>;
    const void *f1 = mode == 1 ? (const void *)k_persistent_ahead<true>
                   : mode == 2 ? (const void *)k_persistent_stamp<true> : (const void *)k_persistent_phase<true>;
    return occupancy_both(f0, f1, block, persistent_lds(mode, block, nc_max), blocks_per_cu);
}

hipError_t launch_gather_params(int32_t n, const int32_t *perm, const double *W, const double *L,
                                const double *V, double *par, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_gather_params, dim3(grid), dim3(256), 0, s, n, perm, W, L, V, par);
    return hipGetLastError();
}

hipError_t launch_colour_phase(const KCirc &kc, const KCall &call, int c, int count,
                               int with_fixed, hipStream_t s) {
    int grid = (count + 255) / 256;
    if (with_fixed) grid = max(grid, min(1024, (kc.n_fixA + kc.n_fixB + 255) / 256));
    grid = max(grid, 1);
    if (junctions(kc)) hipLaunchKernelGGL(k_colour_phase<true>, dim3(grid), dim3(256), 0, s, kc, call, c, with_fixed);
    else hipLaunchKernelGGL(k_colour_phase<false>, dim3(grid), dim3(256), 0, s, kc, call, c, with_fixed);
    return hipGetLastError();
}

hipError_t launch_fixed(const KCirc &kc, const KCall &call, hipStream_t s) {
    const int grid = std::max(1, std::min(1024, (kc.n_fixA + kc.n_fixB + 255) / 256));
    hipLaunchKernelGGL(k_fixed, dim3(grid), dim3(256), 0, s, kc, call);
    return hipGetLastError();
}

hipError_t launch_linear_add(int32_t n, const int32_t *idx, const double *val, double *A, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_linear_add, dim3((n + 255) / 256), dim3(256), 0, s, n, idx, val, A);
    return hipGetLastError();
}

hipError_t launch_newton_update(int32_t n, int32_t n_clamp, const uint8_t *clamp, const double *y, double *x,
                                double vstep,
                                unsigned long long *step_bits, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_newton_update, dim3((n + 255) / 256), dim3(256), 0, s, n, n_clamp, clamp, y, x, vstep,
                       step_bits);
    return hipGetLastError();
}

hipError_t launch_hub(const KCirc &kc, const KCall &call, hipStream_t s) {
    if (kc.n_hub == 0) return hipSuccess;
    const int grid = min((kc.n_hub_chunks + 3) / 4, 4096);
    hipLaunchKernelGGL(k_hub, dim3(grid), dim3(256), 0, s, kc, call);
    return hipGetLastError();
}

hipError_t launch_persistent(const KCirc &kc, const KCall &call, const KSync &ks,
                             const double *buf, int mode, int grid, int block, bool cooperative,
                             hipStream_t s, int n_part, int n_global_chunks, const KLocal &kl) {
    KCirc a = kc;
    KCall b = call;
    KSync c = ks;
    const double *d = buf;
    int np = n_part, ng = n_global_chunks;
    KLocal l = kl;
    void *args[] = {&a, &b, &c, &d, &np, &ng, &l};
    const bool J = junctions(kc);
    const void *fn = mode == 1 ? (kl.n == 0 && n_part == grid
                                      ? (J ? (const void *)k_persistent_ahead_single<true>
                                           : (const void *)k_persistent_ahead_single<false>)
                                      : (J ? (const void *)k_persistent_ahead<true>
                                           : (const void *)k_persistent_ahead<false>))
                   : mode == 2 ? (J ? (const void *)k_persistent_stamp<true> : (const void *)k_persistent_stamp<false>)
                               : (J ? (const void *)k_persistent_phase<true> : (const void *)k_persistent_phase<false>);
    const size_t shm = persistent_lds(mode, block, kc.nc_max);
    if (!cooperative) return hipLaunchKernel(fn, dim3(grid), dim3(block), args, shm, s);
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, shm, s);
}

hipError_t launch_eval_buffer(const KCirc &kc, const KCall &call, double *buf, hipStream_t s) {
    if (kc.n == 0) return hipSuccess;
    const int grid = (kc.n + 255) / 256;
    if (junctions(kc)) hipLaunchKernelGGL(k_eval_buffer<true>, dim3(grid), dim3(256), 0, s, kc, call, buf);
    else hipLaunchKernelGGL(k_eval_buffer<false>, dim3(grid), dim3(256), 0, s, kc, call, buf);
    return hipGetLastError();
}

size_t region_lds_bytes(int lds_int, int nc_max, int block) {
    return sizeof(double) * ((size_t)lds_int + (size_t)nc_max * block);
}

hipError_t region_capacity(int block, int lds_int, int nc_max, int *blocks_per_cu) {
    return occupancy_both((const void *)k_region<false>, (const void *)k_region<true>, block,
                          region_lds_bytes(lds_int, nc_max, block), blocks_per_cu);
}

// After a region launch: large shared entries, then the hub sums over their parts.
static hipError_t launch_region_followups(const KCirc &kc, const KCall &call, const KRegion &kr, hipStream_t s) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t n_fold = (kr.n_deferred + FOLD_E - 1) / FOLD_E;
    if (n_fold + kc.n_hub > 0) {
        hipLaunchKernelGGL(k_region_tail, dim3(n_fold + kc.n_hub), dim3(256), 0, s, kc, call, kr, n_fold);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_region(const KCirc &kc, const KCall &call, const KRegion &kr, int block, hipStream_t s) {
    const int grid = std::max(kr.n_regions, 1);
    const size_t shm = region_lds_bytes(kr.lds_int, kr.nc_max, block);
    if (junctions(kc)) hipLaunchKernelGGL(k_region<true>, dim3(grid), dim3(block), shm, s, kc, call, kr);
    else hipLaunchKernelGGL(k_region<false>, dim3(grid), dim3(block), shm, s, kc, call, kr);
    return launch_region_followups(kc, call, kr, s);
}

hipError_t region_grid_capacity(int block, int lds_int, int nc_max, int *blocks_per_cu) {
    return occupancy_both((const void *)k_region_grid<false>, (const void *)k_region_grid<true>, block,
                          region_lds_bytes(lds_int, nc_max, block), blocks_per_cu);
}

hipError_t launch_region_grid(const KCirc &kc, const KCall &call, const KRegion &kr, const KSync &ks, int block,
                              bool cooperative, hipStream_t s) {
    KCirc a = kc;
    KCall b = call;
    KRegion r = kr;
    KSync k = ks;
    void *args[] = {&a, &b, &r, &k};
    const int grid = std::max(kr.n_regions, 1);
    const size_t shm = region_lds_bytes(kr.lds_int, kr.nc_max, block);
    const void *fn = junctions(kc) ? (const void *)k_region_grid<true> : (const void *)k_region_grid<false>;
    hipError_t e = cooperative ? hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, shm, s)
                               : hipLaunchKernel(fn, dim3(grid), dim3(block), args, shm, s);
    if (e != hipSuccess) return e;
    return launch_region_followups(kc, call, kr, s);
}

hipError_t launch_permute_rows(int32_t n, const int32_t *idx, const double *src, int32_t n_src, int32_t rows,
                               double *dst, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_rows, dim3((n + 255) / 256), dim3(256), 0, s, n, idx, src, n_src, rows, dst);
    return hipGetLastError();
}

hipError_t launch_dev_const(const KCirc &kc, double *sdp, hipStream_t s) {
    if (kc.n == 0) return hipSuccess;
    const int grid = std::max(1, std::min(8192, (kc.n + 255) / 256));
    hipLaunchKernelGGL(k_dev_const, dim3(grid), dim3(256), 0, s, kc, sdp);
    return hipGetLastError();
}

hipError_t launch_serial(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows, double *buf,
                         const int32_t *ipos, hipStream_t s) {
    const int64_t tot = nnz + n_rows;
    const int gz = (int)std::min<int64_t>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_zero, dim3(std::max(gz, 1)), dim3(256), 0, s, call.A, nnz, call.b, n_rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_eval_buffer(kc, call, buf, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_serial_stamp, dim3(1), dim3(64), 0, s, kc, call, buf, ipos);
    return hipGetLastError();
}

hipError_t launch_atomic_wave(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows, hipStream_t s) {
    const int64_t tot = nnz + n_rows;
    const int gz = (int)std::min<int64_t>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_zero, dim3(std::max(gz, 1)), dim3(256), 0, s, call.A, nnz, call.b, n_rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int grid = (kc.n + 255) / 256;
    grid = std::max(grid, std::min(1024, (kc.n_fixA + kc.n_fixB + 255) / 256));
    if (junctions(kc)) hipLaunchKernelGGL(k_atomic_wave<true>, dim3(std::max(grid, 1)), dim3(256), 0, s, kc, call);
    else hipLaunchKernelGGL(k_atomic_wave<false>, dim3(std::max(grid, 1)), dim3(256), 0, s, kc, call);
    return hipGetLastError();
}

hipError_t launch_atomic(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows,
                         hipStream_t s) {
    const int64_t tot = nnz + n_rows;
    const int gz = (int)std::min<int64_t>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_zero, dim3(std::max(gz, 1)), dim3(256), 0, s, call.A, nnz, call.b, n_rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int grid = (kc.n + 255) / 256;
    grid = std::max(grid, std::min(1024, (kc.n_fixA + kc.n_fixB + 255) / 256));
    if (junctions(kc)) hipLaunchKernelGGL(k_atomic<true>, dim3(std::max(grid, 1)), dim3(256), 0, s, kc, call);
    else hipLaunchKernelGGL(k_atomic<false>, dim3(std::max(grid, 1)), dim3(256), 0, s, kc, call);
    return hipGetLastError();
}

}  // namespace cs
