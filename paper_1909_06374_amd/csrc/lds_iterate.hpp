// lds_iterate.hpp -- the light-curve iteration (Sec. 2.1, Sec. 3.2.2) for a
// curve that fits in one workgroup's LDS: the whole loop runs inside one
// kernel, one workgroup per curve, and HBM is touched only to read the fixed
// per-curve tables (sorted draw, its log10, target moduli, twiddles) and to
// write the result.
//
// Per iteration, inside LDS:
//   forward FFT of z[m] = x[2m] + i x[2m+1]  ->  fold to the real spectrum,
//   replace moduli, unfold  ->  inverse FFT gives y  ->  block radix sort of
//   (key(y[n]), n)  ->  for sorted position k holding sample n:
//   rank[n] = k, x[n] = s[k]  ->  delta of Eq. 4 from the log10 table.
//
// LDS layout (bytes): [work: FFT buffer / sort keys / sort counters]
//                     [ibuf: N uint16 sorted indices] [rank: N uint16]
//                     [scratch: 64 words + 40 doubles]
#pragma once
#include "common.hpp"
#include "lds_fft.hpp"
#include "lds_sort.hpp"

namespace agn {

// One curve handled by the LDS-resident kernels.
struct LcDesc {
    int32_t n;             // real length N
    int32_t iters;         // iterations to run
    double tol;            // stopping rule (see agn_lc_iterate)
    const void* amp;       // T[N/2 + 1] target moduli
    const double* x0;      // [N] PDF draw, draw order
    double* s64;           // [N] sorted draw (written by the prep kernel)
    void* sT;              // T[N] sorted draw in working precision
    double* L;             // [N] log10 of the sorted draw
    uint32_t* rank0;       // [N] rank of x0[n] in the sorted draw
    int32_t* valid;        // 1 if every draw value is finite and > 0
    double* x_out;         // [N]
    double* delta_out;     // [iters] or null
    int32_t* iters_done;   // [1] or null
    uint32_t* rank_out;    // [N] or null
    const void* tw;        // cplx<double>[N/2 + 1], W_N^t
    FftPlan plan;          // radices of the length-N/2 complex FFT
};

// LDS bytes of the iteration kernel (host and device agree on this layout).
template <typename T>
__host__ __device__ inline size_t lds_iter_layout(int N, int nt, size_t* ibuf_off, size_t* rank_off,
                                                   size_t* scratch_off, size_t* tw_off = nullptr) {
    typedef typename key_of<T>::type K;
    size_t work = sort_keys_bytes<K>(N);
    const size_t fft = (size_t)cpad_size<T>(N / 2) * sizeof(cplx<T>);
    if (fft > work) work = fft;
    const size_t cnt = sort_cnt_bytes(nt);
    if (cnt > work) work = cnt;
    work = (work + 15) & ~(size_t)15;
    const size_t ib = work;
    const size_t rk = ib + ((sort_ibuf_bytes(N) + 15) & ~(size_t)15);
    const size_t sc = rk + (((size_t)N * 2 + 15) & ~(size_t)15);
    const size_t tw = sc + 128 * 4 + 64 * 8;
    if (ibuf_off) *ibuf_off = ib;
    if (rank_off) *rank_off = rk;
    if (scratch_off) *scratch_off = sc;
    if (tw_off) *tw_off = tw;
    return tw + (size_t)tw_lds_entries(N) * sizeof(cplx<double>);
}

__host__ __device__ inline size_t lds_prep_layout(int N, int nt, size_t* scratch_off) {
    size_t work = sort_keys_bytes<uint64_t>(N);
    const size_t cnt = sort_cnt_bytes(nt);
    if (cnt > work) work = cnt;
    if (sort_ibuf_bytes(N) > work) work = sort_ibuf_bytes(N);
    work = (work + 15) & ~(size_t)15;
    if (scratch_off) *scratch_off = work;
    return work + 128 * 4;
}

// Value of x in lane l (l uniform over the wave).
AGN_DEV uint32_t read_lane(uint32_t x, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)x, l); }
AGN_DEV double read_lane(double x, int l) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Deterministic sum over a group of threads (fixed butterfly + fixed wave
// order); (tid, nt) as for block_radix_sort.  Every thread of the workgroup
// calls it (it holds workgroup barriers).
template <typename V>
AGN_DEV V block_sum(V v, V* scratch /* >= 64 */, int tid, int nt) {
    const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
    __syncthreads();
    if (nt < 64) {
        // Partial single wave: serial sum in thread order.
        scratch[tid] = v;
        __syncthreads();
        V t = scratch[0];
        for (int i = 1; i < nt; ++i) t += scratch[i];
        __syncthreads();
        return t;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) scratch[wave] = v;
    __syncthreads();
    // lane w loads wave w's partial (one load per lane, no waits in a loop);
    // the partials are then added in wave order from the lanes
    const V s = lane < nw ? scratch[lane] : V(0);
    V t = read_lane(s, 0);
#pragma unroll
    for (int w = 1; w < 16; ++w)
        if (w < nw) t += read_lane(s, w);
    __syncthreads();
    return t;
}

// Two-level FP64 twiddle table of length N in LDS at `at` (tw_lds_entries(N)
// entries), filled from the half table tg[t] = W_N^t, t <= N/2.  All threads
// of the block take part; the caller's next barrier publishes the table.
AGN_DEV TwLds lds_load_twiddles(unsigned char* at, const cplx<double>* __restrict__ tg, int N, int tid, int nt) {
    const int M = N / 2;
    TwLds tw;
    tw.bits = tw_lds_bits(N);
    cplx<double>* lo = (cplx<double>*)at;
    cplx<double>* hi = lo + (1 << tw.bits);
    const int nlo = 1 << tw.bits, nhi = (N + nlo - 1) / nlo;
    for (int u = tid; u < nlo + nhi; u += nt) {
        int t = u < nlo ? u : (u - nlo) * nlo;
        // nlo <= N/2 + 1 entries of the half table exist for every N >= 2
        cplx<double> w;
        if (t <= M) {
            w = tg[t];
        } else {
            const cplx<double> v = tg[t - M];  // W_N^{t} = -W_N^{t - N/2}
            w = cmk(-v.re, -v.im);
        }
        if (u < nlo) lo[u] = w;
        else hi[u - nlo] = w;
    }
    tw.lo = lo;
    tw.hi = hi;
    return tw;
}

// Stable ascending ranking of the N = IPT * blockDim.x real values y held in
// LDS at Zf[rpad(p)] (the inverse transform's output): on return
// ibuf[hpad(k)] is the sample index at sorted position k, ties by index.
// (tid, nt): the curve's threads (see block_radix_sort).
// FP64: keys are the order-preserving integer images of y.  FP32 form: keys
// are y mapped in FP64 onto 2^30 levels over [min y, max y] (rounded toward
// zero).  The map is non-decreasing, not strictly increasing: two values
// closer than its step, range * 2^-30, can share a key and are then ordered
// by index.  That step lies far below the FP32 round-off of the transforms,
// and 30-bit keys take 6 radix passes instead of 7.  Every thread of the
// workgroup calls this; it overwrites the LDS work region from `smem` on.
template <typename T, int IPT>
AGN_DEV void lds_rank_series(const T* Zf, unsigned char* smem, uint16_t* ibuf, uint32_t* scratch, int tid,
                             int nt) {
    typedef typename key_of<T>::type K;
    K key[IPT];
    uint32_t idx2[IPT / 2];
    const int tk = opaque(tid);
    if constexpr (sizeof(T) == 4) {
        float y[IPT];
        float mn = Zf[rpad<T>(tk * IPT)], mx = mn;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            y[i] = Zf[rpad<T>(tk * IPT + i)];
            mn = fminf(mn, y[i]);
            mx = fmaxf(mx, y[i]);
        }
        // block min / max (the block is a power of two: one partial
        // wave, or whole waves)
        float* fs = (float*)scratch;  // free until the sort below (barrier before it)
        if (nt < 64) {
            fs[tid] = mn;
            fs[32 + tid] = mx;
            __syncthreads();
            for (int w = 0; w < nt; ++w) {
                mn = fminf(mn, fs[w]);
                mx = fmaxf(mx, fs[32 + w]);
            }
        } else {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                mn = fminf(mn, __shfl_xor(mn, o, 64));
                mx = fmaxf(mx, __shfl_xor(mx, o, 64));
            }
            const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: no VGPR to keep
            if ((tid & 63) == 0) {
                fs[wv] = mn;
                fs[32 + wv] = mx;
            }
            __syncthreads();
            // lane w loads wave w's extremes (lanes past the last wave
            // repeat wave 0's), then the same butterfly across lanes
            const int l = (tid & 63) < (nt >> 6) ? (tid & 63) : 0;
            mn = fs[l];
            mx = fs[32 + l];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                mn = fminf(mn, __shfl_xor(mn, o, 64));
                mx = fmaxf(mx, __shfl_xor(mx, o, 64));
            }
        }
        const double lo = (double)mn, rng = (double)mx - lo;
        const double sc = rng > 0.0 ? 1073741823.0 / rng : 0.0;
#pragma unroll
        for (int i = 0; i < IPT; ++i) key[i] = (K)fmin(((double)y[i] - lo) * sc, 1073741823.0);
    } else {
#pragma unroll
        for (int i = 0; i < IPT; ++i) key[i] = ord_key(Zf[rpad<T>(tk * IPT + i)]);
    }
#pragma unroll
    for (int j = 0; j < IPT / 2; ++j)
        idx2[j] = (uint32_t)(tk * IPT + 2 * j) | ((uint32_t)(tk * IPT + 2 * j + 1) << 16);
    __syncthreads();
    // FP32 form: indices < N <= 2^14 ride in the key word for the last passes
    block_radix_sort<K, IPT, true, sizeof(T) == 4 ? 30 : 8 * (int)sizeof(K), sizeof(T) == 4 ? 14 : 0>(
        key, idx2, smem, ibuf, scratch, tid, nt);
}

// One-time preparation of one curve: stable argsort of the draw (64-bit
// keys), sorted tables and starting ranks.  (tid, nt): the curve's threads
// (the workgroup, or an aligned run of whole waves of it) with the LDS region
// at smem; every thread of the workgroup calls this.  writes = false: compute
// only (a workgroup slot without a curve of its own).
template <typename T, int E>
AGN_DEV void lds_prep_curve(const LcDesc& d, unsigned char* smem, int tid, int nt, bool writes) {
    constexpr int IPT = 2 * E;
    const int N = d.n;
    size_t sc_off;
    lds_prep_layout(N, nt, &sc_off);
    uint32_t* scratch = (uint32_t*)(smem + sc_off);
    uint16_t* ibuf = (uint16_t*)smem;  // aliases the sort work region

    uint64_t key[IPT];
    uint32_t idx2[IPT / 2];
    int bad = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = tid * IPT + i;
        const double x = d.x0[p];
        bad |= !(x > 0.0 && x <= 1.7976931348623157e308);
        key[i] = ord_key(x);
    }
#pragma unroll
    for (int j = 0; j < IPT / 2; ++j)
        idx2[j] = (uint32_t)(tid * IPT + 2 * j) | ((uint32_t)(tid * IPT + 2 * j + 1) << 16);
    // any invalid value among this curve's threads (the sort's first use of
    // scratch comes after a barrier, so the flag word is read before it)
    if (tid == 0) scratch[0] = 0u;
    __syncthreads();
    if (bad) atomicOr(&scratch[0], 1u);
    __syncthreads();
    bad = (int)scratch[0];
    block_radix_sort<uint64_t, IPT, false>(key, idx2, smem, ibuf, scratch, tid, nt);
    if (!writes) return;
    T* sT = (T*)d.sT;
#pragma unroll 4
    for (int u = 0; u < IPT; ++u) {
        const int k = u * nt + tid;
        const uint32_t src = ibuf[hpad(k)];
        const double v = d.x0[src];
        d.s64[k] = v;
        sT[k] = (T)v;
        d.L[k] = log10(v);
        d.rank0[src] = (uint32_t)k;
    }
    if (tid == 0) *d.valid = bad ? 0 : 1;
}

// Same block shape as the iteration kernel; one workgroup per curve.
template <typename T, int E>
__global__ __launch_bounds__(1024) void k_lds_prep(const LcDesc* __restrict__ descs) {
    extern __shared__ __align__(16) unsigned char smem[];
    lds_prep_curve<T, E>(descs[blockIdx.x], smem, threadIdx.x, blockDim.x, true);
}

// The iteration of one curve (Sec. 2.1, Sec. 3.2.2) in LDS.  FUSE2: the plan
// ends with radix 2 (the host checks), and the forward transform's last pass
// is fused with the replacement (lds_fold_replace_r2).  (tid, nt, smem,
// writes) as for lds_prep_curve.  The loop runs max_iters >= d.iters trips so
// that curves sharing a workgroup meet the same barriers; a curve that has
// done its iterations, stopped, or holds an invalid draw keeps computing but
// changes and writes nothing.  solo: the curve has the workgroup to itself
// (an invalid draw then returns at once).
template <typename T, int E, bool FUSE2>
AGN_DEV void lds_iterate_curve(const LcDesc& d, unsigned char* smem, int tid, int nt, bool writes, int max_iters,
                               bool solo) {
    constexpr int IPT = 2 * E;
    const int N = d.n, M = N / 2;
    const bool valid = *d.valid != 0;
    if (solo && !valid) {
        if (tid == 0 && d.iters_done && writes) *d.iters_done = -1;
        return;
    }

    size_t ib_off, rk_off, sc_off, tw_off;
    lds_iter_layout<T>(N, nt, &ib_off, &rk_off, &sc_off, &tw_off);
    cplx<T>* Zc = (cplx<T>*)smem;
    T* Zf = (T*)smem;
    uint16_t* ibuf = (uint16_t*)(smem + ib_off);
    uint16_t* rank16 = (uint16_t*)(smem + rk_off);
    uint32_t* scratch = (uint32_t*)(smem + sc_off);
    double* dscratch = (double*)(smem + sc_off + 128 * 4);

    const gmem<T>* __restrict__ amp = as_global((const T*)d.amp);
    const gmem<T>* __restrict__ sT = as_global((const T*)d.sT);
    const gmem<double>* __restrict__ s64 = as_global(d.s64);
    const gmem<double>* __restrict__ L = as_global(d.L);
    const gmem<uint32_t>* __restrict__ rank0 = as_global(d.rank0);
    const TwLds tw = lds_load_twiddles(smem + tw_off, (const cplx<double>*)d.tw, N, tid, nt);
    const FftPlan& plan = d.plan;  // read in place (uniform loads), not copied to private memory

#pragma unroll 4
    for (int u = 0; u < IPT; ++u) {
        const int p = u * nt + tid;
        const uint32_t r = rank0[p];
        rank16[p] = (uint16_t)r;
        Zf[rpad<T>(p)] = sT[r];
    }
    __syncthreads();

    // the stopping rule is the batch's (one tol for every curve)
    const bool stop_rule = d.tol >= 0.0;
    bool active = valid && d.iters > 0;
    int done = 0;
#pragma unroll 1
    for (int it = 0; it < max_iters; ++it) {
        if (stop_rule && !solo && !__syncthreads_or(active ? 1 : 0)) break;
        if constexpr (FUSE2) {
            // the last forward pass (radix 2) runs inside the replacement
            lds_fft_passes<T, E, false>(Zc, M, plan, 0, plan.npass - 1, 1, tid, nt, tw);
            lds_fold_replace_r2<T>(Zc, M, amp, tw, tid, nt);
            lds_fft<T, E, true>(Zc, M, plan, tid, nt, tw);
        } else {
            lds_fft<T, E, false>(Zc, M, plan, tid, nt, tw);
            lds_fold_replace<T>(Zc, M, amp, tw, tid, nt);
            lds_fft<T, E, true>(Zc, M, plan, tid, nt, tw);
        }

        lds_rank_series<T, IPT>(Zf, smem, ibuf, scratch, tid, nt);

        // x_i[t] = s[k]; Eq. 4 terms from the log10 table.  The exact
        // fixed-point test (values equal, not only ranks) matters only to the
        // stopping rule, so the sorted draw is read only when tol >= 0.
        // Groups of G positions; in each, all LDS lookups first, then all
        // table loads (issued together), then the updates.  A sample whose
        // rank did not change adds an exact zero.
        double acc = 0.0;
        uint32_t chg = 0;
        const int tpost = opaque(tid);
        constexpr int HALF = (IPT % 4 == 0) ? 4 : 2;  // positions per group
#pragma unroll
        for (int h = 0; h < IPT / HALF; ++h) {
            uint32_t tr[HALF];
            double lk[HALF], lr[HALF];
            T sv[HALF];
#pragma unroll
            for (int u = 0; u < HALF; ++u) {
                const uint32_t k = (uint32_t)((h * HALF + u) * nt + tpost);
                const uint32_t t = ibuf[hpad(k)];
                tr[u] = t | ((uint32_t)rank16[t] << 16);
            }
#pragma unroll
            for (int u = 0; u < HALF; ++u) {
                const uint32_t k = (uint32_t)((h * HALF + u) * nt + tpost);
                lk[u] = L[k];
                lr[u] = L[tr[u] >> 16];
                sv[u] = sT[k];
            }
#pragma unroll
            for (int u = 0; u < HALF; ++u) {
                const uint32_t k = (uint32_t)((h * HALF + u) * nt + tpost);
                const uint32_t t = tr[u] & 0xFFFFu, ro = tr[u] >> 16;
                if (active) {
                    rank16[t] = (uint16_t)k;
                    Zf[rpad<T>(t)] = sv[u];
                }
                const double dl = lk[u] - lr[u];
                acc += dl * dl;
                if (stop_rule && ro != k) chg += (s64[k] != s64[ro]) ? 1u : 0u;
            }
        }
        acc = block_sum<double>(acc, dscratch, tid, nt);
        const double delta = sqrt(acc / (double)N);
        if (active) {
            if (tid == 0 && d.delta_out && writes) d.delta_out[it] = delta;
            done = it + 1;
        }
        if (stop_rule) {
            chg = block_sum<uint32_t>(chg, scratch + 64, tid, nt);
            if (chg == 0u || (d.tol > 0.0 && delta <= d.tol)) {
                active = false;
                if (solo) break;
            }
        }
        if (it + 1 >= d.iters) active = false;
    }
    __syncthreads();
    if (!writes) return;
    if (!valid) {
        if (tid == 0 && d.iters_done) *d.iters_done = -1;
        return;
    }
#pragma unroll 4
    for (int u = 0; u < IPT; ++u) {
        const int p = u * nt + tid;
        const uint32_t r = rank16[p];
        d.x_out[p] = s64[r];
        if (d.rank_out) d.rank_out[p] = r;
    }
    if (tid == 0) {
        if (d.iters_done) *d.iters_done = done;
        if (d.delta_out)
            for (int j = done; j < d.iters; ++j) d.delta_out[j] = 0.0;
    }
}

// One workgroup per curve.
template <typename T, int E, bool FUSE2>
__global__ __launch_bounds__(1024) void k_lds_iterate(const LcDesc* __restrict__ descs) {
    extern __shared__ __align__(16) unsigned char smem[];
    const LcDesc& d = descs[blockIdx.x];
    lds_iterate_curve<T, E, FUSE2>(d, smem, threadIdx.x, blockDim.x, true, d.iters, true);
}

// ----------------------------------------------------------------------------
// Every LDS-resident curve of a batch, whatever its length, in one persistent
// launch.  Work items are packs: the curves of one length that fill a
// 1024-thread workgroup (1024 / nt of them, nt = N / IPT threads each, every
// curve's threads an aligned run of whole waves, each curve its own LDS
// region of `stride` bytes); the last pack of a length may hold fewer, and
// its empty slots compute on a copy of the pack's first curve without
// writing.  The packs are ordered longest first and the persistent
// workgroups take them in grid-stride order.  Each pack runs the one-time
// preparation and then the iteration, with the same per-curve code and
// arithmetic as k_lds_prep / k_lds_iterate, so results are bit-identical.
// ----------------------------------------------------------------------------
struct LdsPack {
    int32_t first;      // first curve (index into the descriptor array)
    int32_t count;      // curves in the pack (<= 1024 / nt)
    int32_t E;          // size class: IPT / 2 (4, 6 or 8)
    int32_t nt;         // threads per curve (a multiple of 64)
    int32_t fuse2;      // the length's plan ends with radix 2
    int32_t max_iters;  // largest iteration count in the pack
    uint32_t stride;    // LDS bytes per curve
    int32_t pad;
};

template <typename T, int E>
AGN_DEV void lds_pack_curve(const LcDesc& d, unsigned char* smem, int tid, int nt, bool real, int max_iters,
                            bool fuse2) {
    lds_prep_curve<T, E>(d, smem, tid, nt, real);
    // the tables written above are read back below by other threads of the
    // workgroup: make them visible first
    __threadfence();
    __syncthreads();
    if (fuse2) lds_iterate_curve<T, E, true>(d, smem, tid, nt, real, max_iters, false);
    else lds_iterate_curve<T, E, false>(d, smem, tid, nt, real, max_iters, false);
}

// grid: persistent workgroups (at most npacks), block 1024, dynamic LDS: the
// largest 1024 / nt * stride of the packs.
template <typename T>
__global__ __launch_bounds__(1024) void k_lds_packs(const LcDesc* __restrict__ descs,
                                                    const LdsPack* __restrict__ packs, int npacks) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int p = blockIdx.x; p < npacks; p += gridDim.x) {
        const LdsPack& pk = packs[p];
        const int nt = pk.nt;
        const int sub = (int)threadIdx.x / nt, tid = (int)threadIdx.x - sub * nt;
        const bool real = sub < pk.count;
        const LcDesc& d = descs[pk.first + (real ? sub : 0)];
        unsigned char* base = smem + (size_t)sub * pk.stride;
        if (pk.E == 8) lds_pack_curve<T, 8>(d, base, tid, nt, real, pk.max_iters, pk.fuse2 != 0);
        else if (pk.E == 6) lds_pack_curve<T, 6>(d, base, tid, nt, real, pk.max_iters, pk.fuse2 != 0);
        else lds_pack_curve<T, 4>(d, base, tid, nt, real, pk.max_iters, pk.fuse2 != 0);
        __syncthreads();  // the next pack reuses the LDS
    }
}

}  // namespace agn
