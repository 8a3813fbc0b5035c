// lds_sort.hpp -- stable least-significant-digit radix sort of one block of
// keys held in registers, used for the per-iteration ranking (32-bit keys of
// float values, 64-bit keys of double values) and for the one-time sort of
// the PDF draw.
//
// Layout: "blocked" -- thread t holds the IPT consecutive positions
// t * IPT + i.  Digits are RB = 5 bits wide.  Ranking uses thread-private
// counters, two 16-bit counters per 32-bit LDS word: digit d lives in word
// (d mod 16) * T + t, half d / 16.  A thread walks its items in position
// order, so the old value of the counter is the number of earlier equal
// digits in the same thread.  One exclusive scan of the words in memory order
// (word lane, then thread) then yields, for each half separately, offsets in
// (digit, thread) order; adding the low-half total to every high half puts
// digits 16..31 after digits 0..15.  Every pass is therefore stable, and so is
// the whole sort.
//
// Packed tail (IB > 0, 32-bit keys): once the key bits still to be sorted and
// an IB-bit index fit in one word, each key is replaced by
// (remaining key bits) << IB | index, and the later passes move that single
// word instead of a key and a separate 16-bit index.
#pragma once
#include "common.hpp"

namespace agn {

// Inclusive scan of one uint32 per lane across a 64-lane wave with DPP
// moves: row shifts by 1, 2, 4, 8 (lanes shifted in from outside the row add
// zero), then the last lane of rows 0 and 2 is added to rows 1 and 3 and the
// last lane of row 1 to rows 2 and 3.  Lanes only read lower lanes, so a
// partial wave scans its active lanes correctly.
AGN_DEV uint32_t wave_inclusive_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Exclusive scan of one uint32 per thread over the block (fixed order).
// One barrier: every wave publishes its total; then lane l of every wave
// loads the total of wave l, and a scan across the lanes gives each wave the
// sum of the totals before it (read from lane wave - 1) and the block total
// (lane nw - 1).  One load per lane instead of a loop that waits for each
// word in turn: right after the barrier every wave is here, so such waits
// would leave the SIMDs idle.  The caller must not overwrite scratch[0 .. nw)
// until every thread has returned (a later barrier).
// (tid, nt): the thread's index within the group of threads that scans, and
// the group's size; a group is a whole workgroup or an aligned run of whole
// waves of it.
AGN_DEV uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch /* >= nw words */,
                                      uint32_t* total, int tid, int nt) {
    const int lane = tid & 63, wave = tid >> 6, nw = (nt + 63) >> 6;
    const uint32_t inc = wave_inclusive_scan(v);
    const int last = (nt - (wave << 6) < 64) ? (nt - (wave << 6) - 1) : 63;
    if (lane == last) scratch[wave] = inc;
    __syncthreads();
    const uint32_t ti = wave_inclusive_scan(lane < nw ? scratch[lane] : 0u);
    const uint32_t pre = wave > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)ti, wave - 1) : 0u;
    if (total) *total = (uint32_t)__builtin_amdgcn_readlane((int)ti, nw - 1);
    return pre + inc - v;
}

constexpr int SORT_RB = 5;
constexpr int SORT_LANES = 1 << (SORT_RB - 1);  // counter words per thread

// Padded LDS indices (one pad slot per 128 or 256 bytes) so that the blocked
// accesses, which stride by IPT elements across lanes, spread over the banks.
template <typename K>
AGN_DEV int kpad(int e) { return e + (e >> (sizeof(K) == 4 ? 5 : 4)); }
AGN_DEV int wpad(int w) { return w + (w >> 5); }
// 16-bit element e of a padded array of 32-bit words:
// 2 * wpad(e >> 1) + (e & 1) = e + 2 * (e >> 6).
AGN_DEV int hpad(int e) { return e + ((e >> 6) << 1); }

template <typename K>
__host__ __device__ inline size_t sort_keys_bytes(int n) {
    return ((size_t)n + (n >> (sizeof(K) == 4 ? 5 : 4)) + 1) * sizeof(K);
}
__host__ __device__ inline size_t sort_cnt_bytes(int nthreads) {
    const int w = SORT_LANES * nthreads;
    return ((size_t)w + (w >> 5) + 1) * 4;
}
__host__ __device__ inline size_t sort_ibuf_bytes(int n) {
    const int w = (n + 1) / 2;
    return ((size_t)w + (w >> 5) + 1) * 4;
}

// Sorts (key, idx) ascending by key, stable in position order.
//   key[IPT]           this thread's keys at positions t*IPT + i
//   idx2[IPT/2]        their 16-bit indices, two per word (low half = even i)
//   work               LDS region of max(sort_keys_bytes<K>(N), sort_cnt_bytes(T))
//                      (counters, keys)
//   ibuf               LDS, sort_ibuf_bytes(N), 4-byte aligned, padded (hpad);
//                      may alias `work` only if SEP == false
//   scratch            LDS, >= 20 words, not aliased
// On return ibuf[hpad(k)] holds the index carried by the k-th smallest key
// (after a barrier).  key[] and idx2[] are left in an unspecified state.
//
// Index arithmetic: when T is a multiple of 32, the counter word of digit
// lane l for thread t, wpad(l T + t), equals l (T + T/32) + (t + t/32); the
// thread's own scan words wpad(16 t + q), q < 16, are 16 t + t/2 + q; and
// when IPT divides the pad period, the read-back addresses of a thread's
// IPT keys and IPT/2 index words are a per-thread base plus i (or j).  The
// addresses are the same as the padded formulas, with fewer instructions.
// Passes after which a 32-bit key and an IB-bit index are packed into one
// word (NPASS: never).
template <typename K, int KBITS, int IB>
constexpr int sort_pack_at() {
    constexpr int NPASS = (KBITS + SORT_RB - 1) / SORT_RB;
    if (IB <= 0 || sizeof(K) != 4) return NPASS;
    for (int j = 1; j < NPASS; ++j)
        if (KBITS - SORT_RB * j + IB <= 32) return j;
    return NPASS;
}

template <typename K, int IPT, bool SEP, bool ALIGNED, int KBITS, int IB>
AGN_DEV void block_radix_sort_impl(K (&key)[IPT], uint32_t (&idx2)[IPT / 2], unsigned char* work,
                                   uint16_t* ibuf, uint32_t* scratch, int tid, int T) {
    static_assert(IPT % 2 == 0, "IPT must be even");
    static_assert(KBITS >= 1 && KBITS <= 8 * (int)sizeof(K), "key bits out of range");
    constexpr int NPASS = (KBITS + SORT_RB - 1) / SORT_RB;
    constexpr int PACK_AT = sort_pack_at<K, KBITS, IB>();
    static_assert(PACK_AT == NPASS || SEP, "the packed tail is built for separate key and index regions");
    static_assert(IB >= 0 && IB <= 16, "indices are 16-bit");
    constexpr bool PACK = PACK_AT < NPASS;
    constexpr int PSH = PACK ? SORT_RB * PACK_AT : 0;  // key bits already sorted when packing
    constexpr int PIB = PACK ? IB : 0;
    constexpr uint32_t IMASK = PACK ? (1u << IB) - 1u : 0u;
    constexpr int KPER = sizeof(K) == 4 ? 32 : 16;  // key pad period
    constexpr bool KFAST = (KPER % IPT) == 0;
    constexpr bool IFAST = (32 % (IPT / 2)) == 0;
    uint32_t* cnt = (uint32_t*)work;
    K* kb = (K*)work;
    const uint32_t* ibuf32 = (const uint32_t*)ibuf;
    const int Tp = T + (T >> 5);

#pragma unroll 1
    for (int pass = 0; pass < NPASS; ++pass) {
        const int t = opaque(tid);
        const int tb = t + (t >> 5);
        // packed words hold the key bits from SORT_RB * PACK_AT up, above the index
        const int shift = pass < PACK_AT ? pass * SORT_RB : PIB + (pass - PACK_AT) * SORT_RB;
#pragma unroll
        for (int l = 0; l < SORT_LANES; ++l) cnt[ALIGNED ? l * Tp + tb : wpad(l * T + t)] = 0u;
        // pos[i]: bits 0..15 running position, bits 16..20 the digit.
        uint32_t pos[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const uint32_t d = (uint32_t)(key[i] >> shift) & (2 * SORT_LANES - 1);
            const int l = (int)(d & (SORT_LANES - 1));
            const int a = ALIGNED ? l * Tp + tb : wpad(l * T + t);
            const uint32_t sh = d & SORT_LANES;  // 0 or 16
            // the counter word is private to this thread: the returned old
            // value is the count of earlier equal digits; atomics issue back
            // to back instead of waiting for each read before the next write
            const uint32_t c = atomicAdd(&cnt[a], 1u << sh);
            pos[i] = ((c >> sh) & 0xFFFFu) | (d << 16);
        }
        __syncthreads();
        {
            const int sb = 16 * t + (t >> 1);  // wpad(16 t + q) - q
            uint32_t w[SORT_LANES];
            uint32_t s = 0;
#pragma unroll
            for (int q = 0; q < SORT_LANES; ++q) {
                w[q] = cnt[sb + q];
                s += w[q];
            }
            uint32_t total;
            uint32_t run = block_exclusive_scan(s, scratch, &total, t, T);
            run += (total & 0xFFFFu) << 16;
#pragma unroll
            for (int q = 0; q < SORT_LANES; ++q) {
                cnt[sb + q] = run;
                run += w[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const uint32_t d = pos[i] >> 16;
            const int l = (int)(d & (SORT_LANES - 1));
            const int a = ALIGNED ? l * Tp + tb : wpad(l * T + t);
            const uint32_t sh = d & SORT_LANES;
            pos[i] = (pos[i] & 0xFFFFu) + ((cnt[a] >> sh) & 0xFFFFu);
        }
        __syncthreads();
        const bool last = (pass == NPASS - 1);
        const int kbase = KFAST ? t * IPT + (t * IPT) / KPER : 0;
        const int ibase = IFAST ? t * (IPT / 2) + (t * (IPT / 2)) / 32 : 0;
        if (SEP) {
            if (PACK && pass >= PACK_AT) {
                // packed word in, packed word out (the last pass keeps the index)
                if (!last) {
#pragma unroll
                    for (int i = 0; i < IPT; ++i) kb[kpad<K>((int)pos[i])] = key[i];
                } else {
#pragma unroll
                    for (int i = 0; i < IPT; ++i) ibuf[hpad((int)pos[i])] = (uint16_t)((uint32_t)key[i] & IMASK);
                }
            } else if (PACK && pass + 1 == PACK_AT) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const uint32_t ix = (i & 1) ? (idx2[i / 2] >> 16) : (idx2[i / 2] & 0xFFFFu);
                    kb[kpad<K>((int)pos[i])] = (K)((((uint32_t)key[i] >> PSH) << PIB) | ix);
                }
            } else if (!last) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    kb[kpad<K>((int)pos[i])] = key[i];
                    ibuf[hpad((int)pos[i])] = (uint16_t)((i & 1) ? (idx2[i / 2] >> 16) : idx2[i / 2]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    ibuf[hpad((int)pos[i])] = (uint16_t)((i & 1) ? (idx2[i / 2] >> 16) : idx2[i / 2]);
            }
            __syncthreads();
            if (!last) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) key[i] = kb[KFAST ? kbase + i : kpad<K>(t * IPT + i)];
                if (!PACK || pass + 1 < PACK_AT) {
#pragma unroll
                    for (int j = 0; j < IPT / 2; ++j)
                        idx2[j] = ibuf32[IFAST ? ibase + j : wpad((t * IPT) / 2 + j)];
                }
                __syncthreads();
            }
        } else {
            if (!last) {
#pragma unroll
                for (int i = 0; i < IPT; ++i) kb[kpad<K>((int)pos[i])] = key[i];
                __syncthreads();
#pragma unroll
                for (int i = 0; i < IPT; ++i) key[i] = kb[KFAST ? kbase + i : kpad<K>(t * IPT + i)];
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < IPT; ++i)
                ibuf[hpad((int)pos[i])] = (uint16_t)((i & 1) ? (idx2[i / 2] >> 16) : idx2[i / 2]);
            __syncthreads();
            if (!last) {
#pragma unroll
                for (int j = 0; j < IPT / 2; ++j) idx2[j] = ibuf32[IFAST ? ibase + j : wpad((t * IPT) / 2 + j)];
                __syncthreads();
            }
        }
    }
}

// IPT 16 is used only with 1024-thread groups (the host checks that the
// group size is a multiple of 32 for it), so only the aligned form is built.
// Keys use their low KBITS bits (all others must be zero).  IB > 0: every
// index is below 2^IB, and the tail passes move packed words (32-bit keys).
// (tid, nt): index within and size of the sorting group of threads (the
// workgroup, or an aligned run of whole waves of it); every thread of the
// workgroup must call this, as it contains workgroup barriers.
template <typename K, int IPT, bool SEP, int KBITS = 8 * (int)sizeof(K), int IB = 0>
AGN_DEV void block_radix_sort(K (&key)[IPT], uint32_t (&idx2)[IPT / 2], unsigned char* work,
                              uint16_t* ibuf, uint32_t* scratch, int tid, int nt) {
    if constexpr (IPT >= 16) {
        block_radix_sort_impl<K, IPT, SEP, true, KBITS, IB>(key, idx2, work, ibuf, scratch, tid, nt);
    } else if constexpr (sizeof(K) == 8) {
        // 64-bit keys (one-time draw sort, FP64 path): one general form keeps
        // register pressure low
        block_radix_sort_impl<K, IPT, SEP, false, KBITS, IB>(key, idx2, work, ibuf, scratch, tid, nt);
    } else {
        if ((nt & 31) == 0)
            block_radix_sort_impl<K, IPT, SEP, true, KBITS, IB>(key, idx2, work, ibuf, scratch, tid, nt);
        else
            block_radix_sort_impl<K, IPT, SEP, false, KBITS, IB>(key, idx2, work, ibuf, scratch, tid, nt);
    }
}

}  // namespace agn
