// rANS entropy coding of an array of 32-bit integers (gfx950): the
// compression stage of a time frame, where every flat integer array is coded
// on its own with frequencies counted for that frame (Sec. 4.1).
//
//  Every kernel codes a batch of arrays: grid dimension y selects the
//  array; an array's symbol count may come from device memory.
//  rs_init      min / max / status words
//  rs_window    (large arrays) zero the whole histogram: it is counted in the
//               same pass as the range, relative to a window of 2^20 symbols
//               centred on the first symbol
//  rs_minmax    grid reduction of the symbol range; for large arrays also
//               the histogram over that window (LDS-private for the 8192
//               symbols around the first one, global atomics for the rest);
//               a symbol outside the window flags the two-pass path
//  rs_clear     zero the histogram over the range (fails if wider than 2^20);
//               for a large array whose window held every symbol, only the
//               offset of the range in the window is set
//  rs_hist      histogram: LDS-private per workgroup when the range fits
//               (8192 bins; eight copies of each bin up to 1024), global
//               atomics otherwise; 16-byte symbol loads
//  rs_freq      one workgroup: number of symbols present, most frequent
//               symbol, scaled frequencies (integer arithmetic, exactly the
//               stated rule), their exclusive scan
//  rs_table     one workgroup: the frequency table compressed for the
//               stream -- per present symbol, in ascending order, the run of
//               absent symbols before it and f - 1 as LEB128 varints --
//               by two scans (the present symbols' ranks, then the pairs'
//               byte offsets); positions and bytes in the histogram's
//               buffer, which no later kernel reads
//  rs_encode    one wavefront per block of B symbols, lane k = coder k; the
//               block is coded backwards round by round (symbols loaded eight
//               rounds at a time, the coding table in LDS for ranges up to
//               2048, division by the frequency as a multiply-high with a
//               precomputed reciprocal); the words a round emits are placed
//               by ballot and prefix popcount in the order coders 63 .. 0
//               push them, into a per-block scratch stack
//  rs_scan      exclusive scan of the blocks' word counts
//  rd_*         the decoder (see below)
//  rs_pack      the stream: header, compressed frequency table, block word offsets,
//               final coder states, every block's stack reversed; nothing is
//               written and the status says TPC_ERR_CAPACITY when the
//               stream (its exact size is reported) does not fit
#include "tpc_internal.hpp"
#include "tpc_rans_dec.hpp"

#define RS_LANES 64
#define RS_HEAD 40
#define RS_LDS_BINS 8192
#define RS_MAGIC 0x534E4152u
#define RS_TAB_LDS 2048     // coding table in LDS up to this range (32 KB)
#define RS_CHUNK 8          // rounds whose symbols are loaded at once

namespace {

struct RsArgs {
    const int32_t *sym;
    int64_t n;             // resolved on the device: min(*n_dev, n_cap), or n_cap
    const int64_t *n_dev;  // optional device symbol count
    int64_t n_cap;
    int32_t L, B, nb;
    int32_t fused;         // range and histogram in one pass (large arrays)
    int32_t *mm;           // [0] min, [1] max, [2] status, [3] table bytes, [4] offset of
                           // the range in counts, [5] a symbol left the window,
                           // [6] the window's centre (device)
    uint32_t *counts;      // [TPC_RANS_MAX_RANGE] histogram, then the table's positions and bytes
    uint4 *fc;             // [TPC_RANS_MAX_RANGE] (frequency, cumulative, reciprocal, shifts)
    uint32_t *wcount;      // [nb] words of each block
    uint32_t *wstart;      // [nb + 1]
    uint32_t *states;      // [nb][64]
    uint16_t *scratch;     // [nb][B] each block's word stack, push order
    uint8_t *out;
    uint64_t cap;
    uint64_t *out_size;
    int32_t *dev_status;
};

// Arrays coded together: grid dimension y selects the array.
struct RsBatch {
    RsArgs a[TPC_RANS_BATCH_MAX];
};

__device__ inline RsArgs rs_job(const RsBatch &Bt) {
    RsArgs A = Bt.a[blockIdx.y];
    if (A.n_dev) {
        const int64_t v = *A.n_dev;
        A.n = v < 0 ? 0 : (v < A.n_cap ? v : A.n_cap);
    } else {
        A.n = A.n_cap;
    }
    A.nb = (int32_t)(A.n > 0 ? (A.n + A.B - 1) / A.B : 0);
    return A;
}

// Range R = max - min + 1 (0 for no symbols).
__device__ inline int64_t rs_range(const RsArgs &A) {
    return A.n > 0 ? (int64_t)A.mm[1] - (int64_t)A.mm[0] + 1 : 0;
}

__global__ void rs_init(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    if (threadIdx.x == 0) {
        A.mm[0] = 0x7fffffff;
        A.mm[1] = (int32_t)0x80000000;
        A.mm[2] = TPC_OK;
        A.mm[3] = 0;
        A.mm[4] = 0;
        A.mm[5] = 0;
        A.mm[6] = A.n > 0 ? A.sym[0] : 0;
    }
}

// The symbols as 16-byte vectors where aligned: head (scalar), body (int4),
// tail (scalar).
struct Vec4Split {
    int64_t head, nv;        // scalars before the first aligned vector, vectors
};
__device__ inline Vec4Split vec4_split(const int32_t *p, int64_t n) {
    Vec4Split v;
    const int64_t mis = (int64_t)(((uintptr_t)p >> 2) & 3);
    v.head = mis ? 4 - mis : 0;
    if (v.head > n) v.head = n;
    v.nv = (n - v.head) / 4;
    return v;
}

// Arrays of at least this many symbols count their histogram in the range
// pass (the whole 2^20-entry histogram is cleared for them).
#define RS_FUSE_MIN (1 << 22)
#define RS_WIN_HALF (TPC_RANS_MAX_RANGE / 2)
#define RS_LDS_HALF (RS_LDS_BINS / 2)

__global__ void __launch_bounds__(TPC_BLOCK) rs_window(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    if (!A.fused) return;
    for (int64_t s = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; s < TPC_RANS_MAX_RANGE;
         s += (int64_t)gridDim.x * TPC_BLOCK)
        A.counts[s] = 0;
}

__global__ void __launch_bounds__(TPC_BLOCK) rs_minmax(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    __shared__ int sh[2][TPC_BLOCK / TPC_WAVE];
    __shared__ uint32_t h[RS_LDS_BINS];
    int lo = 0x7fffffff, hi = (int)0x80000000;
    const Vec4Split V = vec4_split(A.sym, A.n);
    const int4 *v4 = reinterpret_cast<const int4 *>(A.sym + V.head);
    const int64_t gtid = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x, G = (int64_t)gridDim.x * TPC_BLOCK;
    // large arrays: counts relative to the window [c - 2^19, c + 2^19) of
    // the first symbol c; the 8192 symbols around c in LDS
    const int64_t c = A.mm[6];
    bool out = false;
    if (A.fused) {
        for (int b = threadIdx.x; b < RS_LDS_BINS; b += TPC_BLOCK) h[b] = 0;
        __syncthreads();
    }
    auto add = [&](int v) {
        const int64_t d = (int64_t)v - c;
        if (d >= -RS_LDS_HALF && d < RS_LDS_HALF) atomicAdd(&h[d + RS_LDS_HALF], 1u);
        else if (d >= -RS_WIN_HALF && d < RS_WIN_HALF) atomicAdd(&A.counts[d + RS_WIN_HALF], 1u);
        else out = true;
    };
    for (int64_t q = gtid; q < V.nv; q += G) {
        const int4 v = v4[q];
        lo = min(lo, min(min(v.x, v.y), min(v.z, v.w)));
        hi = max(hi, max(max(v.x, v.y), max(v.z, v.w)));
        if (A.fused) {
            add(v.x);
            add(v.y);
            add(v.z);
            add(v.w);
        }
    }
    for (int64_t i = gtid; i < V.head + (A.n - V.head - 4 * V.nv); i += G) {
        const int64_t j = i < V.head ? i : V.head + 4 * V.nv + (i - V.head);
        const int v = A.sym[j];
        lo = min(lo, v);
        hi = max(hi, v);
        if (A.fused) add(v);
    }
    if (A.fused) {
        if (out) A.mm[5] = 1;
        __syncthreads();
        for (int b = threadIdx.x; b < RS_LDS_BINS; b += TPC_BLOCK)
            if (h[b]) atomicAdd(&A.counts[b - RS_LDS_HALF + RS_WIN_HALF], h[b]);
    }
#pragma unroll
    for (int d = TPC_WAVE / 2; d > 0; d >>= 1) {
        lo = min(lo, __shfl_xor(lo, d, TPC_WAVE));
        hi = max(hi, __shfl_xor(hi, d, TPC_WAVE));
    }
    const int wid = threadIdx.x / TPC_WAVE;
    if ((threadIdx.x & (TPC_WAVE - 1)) == 0) {
        sh[0][wid] = lo;
        sh[1][wid] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < TPC_BLOCK / TPC_WAVE; ++w) {
            lo = min(lo, sh[0][w]);
            hi = max(hi, sh[1][w]);
        }
        if (lo <= hi) {                     // a workgroup that saw no symbol adds nothing
            atomicMin(&A.mm[0], lo);
            atomicMax(&A.mm[1], hi);
        }
    }
}

// The histogram of a large array counted in its window: the range's offset
// in it (read by rs_freq), unless a symbol left the window.
__device__ inline bool rs_windowed(const RsArgs &A) { return A.fused && A.mm[5] == 0; }

__global__ void __launch_bounds__(TPC_BLOCK) rs_clear(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    const int64_t R = rs_range(A);
    if (R > TPC_RANS_MAX_RANGE) {
        if (blockIdx.x == 0 && threadIdx.x == 0) A.mm[2] = TPC_ERR_ARG;
        return;
    }
    if (rs_windowed(A)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && A.n > 0)
            A.mm[4] = (int32_t)((int64_t)A.mm[0] - ((int64_t)A.mm[6] - RS_WIN_HALF));
        return;
    }
    for (int64_t s = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; s < R; s += (int64_t)gridDim.x * TPC_BLOCK)
        A.counts[s] = 0;
}

// Up to RS_COPY_BINS symbols, each bin has RS_COPIES copies side by side in
// LDS and lane k counts into copy k mod RS_COPIES: a peaked distribution
// sends most lanes of an instruction to a few bins, and the copies spread
// those atomics over banks.
#define RS_COPIES 8
#define RS_COPY_BINS (RS_LDS_BINS / RS_COPIES)
__global__ void __launch_bounds__(TPC_BLOCK) rs_hist(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    __shared__ uint32_t h[RS_LDS_BINS];
    const int64_t R = rs_range(A);
    if (R > TPC_RANS_MAX_RANGE || rs_windowed(A)) return;
    if ((int64_t)blockIdx.x * TPC_BLOCK * 4 >= A.n) return;     // no symbols for this workgroup
    const int lo = A.mm[0];
    const int mode = R <= RS_COPY_BINS ? 2 : (R <= RS_LDS_BINS ? 1 : 0);
    const int cp = mode == 2 ? (threadIdx.x & (RS_COPIES - 1)) : 0;
    const int stride = mode == 2 ? RS_COPIES : 1;
    if (mode) {
        for (int s = threadIdx.x; s < RS_LDS_BINS; s += TPC_BLOCK) h[s] = 0;
        __syncthreads();
    }
    const Vec4Split V = vec4_split(A.sym, A.n);
    const int4 *v4 = reinterpret_cast<const int4 *>(A.sym + V.head);
    const int64_t gtid = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x, G = (int64_t)gridDim.x * TPC_BLOCK;
    auto add = [&](int v) {
        const uint32_t s = (uint32_t)((int64_t)v - lo);
        if (mode) atomicAdd(&h[s * stride + cp], 1u);
        else atomicAdd(&A.counts[s], 1u);
    };
    for (int64_t q = gtid; q < V.nv; q += G) {
        const int4 v = v4[q];
        add(v.x);
        add(v.y);
        add(v.z);
        add(v.w);
    }
    for (int64_t i = gtid; i < V.head + (A.n - V.head - 4 * V.nv); i += G)
        add(A.sym[i < V.head ? i : V.head + 4 * V.nv + (i - V.head)]);
    if (mode) {
        __syncthreads();
        for (int s = threadIdx.x; s < R; s += TPC_BLOCK) {
            uint32_t c = 0;
            for (int k = 0; k < stride; ++k) c += h[s * stride + k];
            if (c) atomicAdd(&A.counts[s], c);
        }
    }
}

// Block-wide reductions for the 1024-thread frequency kernel.
#define RS_FREQ_THREADS 1024
__device__ inline long long rs_block_sum(long long v, long long *sh) {
#pragma unroll
    for (int d = TPC_WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, TPC_WAVE);
    const int wid = threadIdx.x / TPC_WAVE;
    __syncthreads();
    if ((threadIdx.x & (TPC_WAVE - 1)) == 0) sh[wid] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < RS_FREQ_THREADS / TPC_WAVE; ++w) t += sh[w];
    return t;
}

// key = count << 32 | (2^32 - 1 - s): the largest key is the most frequent
// symbol, the smallest s among equals
__device__ inline unsigned long long rs_block_max(unsigned long long v, unsigned long long *sh) {
#pragma unroll
    for (int d = TPC_WAVE / 2; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(v, d, TPC_WAVE);
        v = o > v ? o : v;
    }
    const int wid = threadIdx.x / TPC_WAVE;
    __syncthreads();
    if ((threadIdx.x & (TPC_WAVE - 1)) == 0) sh[wid] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < RS_FREQ_THREADS / TPC_WAVE; ++w) t = sh[w] > t ? sh[w] : t;
    return t;
}

__global__ void __launch_bounds__(RS_FREQ_THREADS) rs_freq(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    const uint32_t *cnt = A.counts + A.mm[4];      // the range's first symbol
    __shared__ long long sh[RS_FREQ_THREADS / TPC_WAVE];
    __shared__ unsigned long long shk[RS_FREQ_THREADS / TPC_WAVE];
    __shared__ int scan_sh[RS_FREQ_THREADS / TPC_WAVE];
    if (A.mm[2] != TPC_OK) return;
    const int64_t R = rs_range(A);
    if (R == 0) return;
    const uint64_t M = 1ull << A.L;
    long long d = 0;
    unsigned long long best = 0;
    for (int64_t s = threadIdx.x; s < R; s += RS_FREQ_THREADS) {
        const uint32_t c = cnt[s];
        d += c > 0;
        const unsigned long long key = ((unsigned long long)c << 32) | (0xffffffffull - (uint64_t)s);
        best = key > best ? key : best;
    }
    const long long D = rs_block_sum(d, sh);
    best = rs_block_max(best, shk);
    if ((uint64_t)D > M) {
        if (threadIdx.x == 0) A.mm[2] = TPC_ERR_ARG;
        return;
    }
    const int64_t sbest = (int64_t)(0xffffffffull - (best & 0xffffffffull));
    long long part = 0;
    for (int64_t s = threadIdx.x; s < R; s += RS_FREQ_THREADS) {
        const uint32_t c = cnt[s];
        const uint32_t f = c ? (uint32_t)((uint64_t)c * (M - (uint64_t)D) / (uint64_t)A.n + 1) : 0u;
        A.fc[s].x = f;
        part += f;
    }
    const long long sum = rs_block_sum(part, sh);
    __syncthreads();
    if (threadIdx.x == 0) A.fc[sbest].x += (uint32_t)((long long)M - sum);
    __threadfence_block();
    __syncthreads();
    // exclusive scan of the frequencies in chunks of the workgroup
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < R; c0 += RS_FREQ_THREADS) {
        const int64_t s = c0 + threadIdx.x;
        const int f = s < R ? (int)A.fc[s].x : 0;
        // block_exclusive_scan covers TPC_BLOCK threads: scan four quarters
        const int lane = threadIdx.x & (TPC_WAVE - 1), wid = threadIdx.x / TPC_WAVE;
        int inc = wave_inclusive_scan(f);
        if (lane == TPC_WAVE - 1) scan_sh[wid] = inc;
        __syncthreads();
        int before = 0, tot = 0;
        for (int w = 0; w < RS_FREQ_THREADS / TPC_WAVE; ++w) {
            const int v = scan_sh[w];
            before += w < wid ? v : 0;
            tot += v;
        }
        __syncthreads();
        if (s < R) {
            A.fc[s].y = carry + (uint32_t)(before + inc - f);
            // floor(x / f) = (t + ((x - t) >> s1)) >> s2, t = mulhi(x, m), for
            // every 32-bit x (division by an invariant integer, Granlund and
            // Montgomery 1994): l = ceil(log2 f), m = floor(2^32 (2^l - f) / f) + 1,
            // s1 = 1, s2 = l - 1; for f = 1, m = 0, s1 = s2 = 0
            uint32_t m = 0, sh = 0;
            if (f > 1) {
                const int l = 32 - __clz(f - 1);
                m = (uint32_t)(((((uint64_t)1 << l) - (uint64_t)f) << 32) / (uint64_t)f + 1);
                sh = 1u | ((uint32_t)(l - 1) << 8);
            }
            A.fc[s].z = m;
            A.fc[s].w = sh;
        }
        carry += (uint32_t)tot;
    }
}

// Compressed frequency table.  The histogram's buffer holds, after the
// frequencies are made, the present symbols in rank order (RS_TAB_POS) and
// the table's bytes (RS_TAB_BYTES on).
#define RS_TAB_BYTES 65536

__device__ inline int varint_len(uint32_t v) { return v < 128u ? 1 : (v < 16384u ? 2 : 3); }

__device__ inline int put_varint(uint8_t *p, uint32_t v) {
    int k = 0;
    while (v >= 0x80u) {
        p[k++] = (uint8_t)(v | 0x80u);
        v >>= 7;
    }
    p[k++] = (uint8_t)v;
    return k;
}

__global__ void __launch_bounds__(TPC_BLOCK) rs_table(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    if (A.mm[2] != TPC_OK) return;
    const int64_t R = rs_range(A);
    uint32_t *pos = A.counts;                                   // [D <= 2^16]
    uint8_t *tb = reinterpret_cast<uint8_t *>(A.counts + RS_TAB_BYTES);
    // ranks of the present symbols
    int D = 0;
    for (int64_t c0 = 0; c0 < R; c0 += TPC_BLOCK) {
        const int64_t s = c0 + threadIdx.x;
        const int present = s < R && A.fc[s].x > 0u;
        int tot;
        const int ex = block_exclusive_scan(present, sh, &tot);
        if (present) pos[D + ex] = (uint32_t)s;
        D += tot;
    }
    __threadfence_block();
    __syncthreads();
    // each pair's bytes at the exclusive scan of the pairs' lengths
    int T = 0;
    for (int c0 = 0; c0 < D; c0 += TPC_BLOCK) {
        const int k = c0 + threadIdx.x;
        uint32_t gap = 0, fm1 = 0;
        int len = 0;
        if (k < D) {
            const uint32_t sk = pos[k];
            gap = sk - (k > 0 ? pos[k - 1] + 1u : 0u);
            fm1 = A.fc[sk].x - 1u;
            len = varint_len(gap) + varint_len(fm1);
        }
        int tot;
        const int ex = block_exclusive_scan(len, sh, &tot);
        if (k < D) {
            const int o = T + ex;
            const int a = put_varint(tb + o, gap);
            put_varint(tb + o + a, fm1);
        }
        T += tot;
    }
    if (threadIdx.x == 0) A.mm[3] = T;
}

// One block of symbols by one wavefront; T is the coding table (LDS or
// global memory, a separate instantiation each so that the loads are not
// generic).
template <class Tab>
__device__ inline void encode_block(const RsArgs &A, Tab T, int b, int lane) {
    const int lo = A.mm[0];
    const int L = A.L;
    const int64_t i0 = (int64_t)b * A.B;
    const int nloc = (int)((i0 + A.B < A.n ? i0 + A.B : A.n) - i0);
    const int32_t *src = A.sym + i0;
    const int rounds = (nloc + RS_LANES - 1) / RS_LANES;
    uint16_t *stack = A.scratch + (size_t)b * A.B;
    uint32_t x = 1u << 16;
    uint32_t top = 0;
    for (int jc = rounds - 1; jc >= 0; jc -= RS_CHUNK) {
        // the symbols of the next RS_CHUNK rounds (coded backwards), loaded together
        int32_t sv[RS_CHUNK];
#pragma unroll
        for (int u = 0; u < RS_CHUNK; ++u) {
            const int k = (jc - u) * RS_LANES + lane;
            sv[u] = (jc - u >= 0 && k < nloc) ? src[k] : lo;
        }
#pragma unroll
        for (int u = 0; u < RS_CHUNK; ++u) {
            const int j = jc - u;
            if (j < 0) break;
            const bool act = j * RS_LANES + lane < nloc;
            const uint4 e = T(act ? (uint32_t)(sv[u] - lo) : 0u);
            const bool emit = act && (uint64_t)x >= ((uint64_t)e.x << (32 - L));
            const unsigned long long mask = __ballot(emit);
            if (emit) {
                // coders above this one push first
                const int rank = __popcll(lane == 63 ? 0ull : mask >> (lane + 1));
                stack[top + rank] = (uint16_t)(x & 0xffffu);
                x >>= 16;
            }
            top += (uint32_t)__popcll(mask);
            if (act) {
                const uint32_t t = __umulhi(x, e.z);
                const uint32_t q = (t + ((x - t) >> (e.w & 0xffu))) >> (e.w >> 8);
                x = (q << L) + (x - q * e.x) + e.y;
            }
        }
    }
    A.states[(size_t)b * RS_LANES + lane] = x;
    if (lane == 0) A.wcount[b] = top;
}

struct LdsTab {
    const uint4 *t;
    __device__ uint4 operator()(uint32_t s) const { return t[s]; }
};
struct GlobalTab {
    const uint4 *__restrict__ t;
    __device__ uint4 operator()(uint32_t s) const { return t[s]; }
};

__global__ void __launch_bounds__(TPC_BLOCK) rs_encode(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    __shared__ uint4 tab[RS_TAB_LDS];
    if (A.mm[2] != TPC_OK) return;                  // uniform over the grid
    const int64_t R = rs_range(A);
    const bool in_lds = R <= RS_TAB_LDS;
    if (in_lds) {
        for (int s = threadIdx.x; s < R; s += TPC_BLOCK) tab[s] = A.fc[s];
        __syncthreads();
    }
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    const int b = blockIdx.x * (TPC_BLOCK / TPC_WAVE) + threadIdx.x / TPC_WAVE;
    if (b >= A.nb) return;                          // after the only barrier
    if (in_lds) encode_block(A, LdsTab{tab}, b, lane);
    else encode_block(A, GlobalTab{A.fc}, b, lane);
}

__global__ void __launch_bounds__(TPC_BLOCK) rs_scan(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    uint32_t carry = 0;
    for (int c0 = 0; c0 < A.nb; c0 += TPC_BLOCK) {
        const int b = c0 + threadIdx.x;
        const int v = (b < A.nb && A.mm[2] == TPC_OK) ? (int)A.wcount[b] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, sh, &tot);
        if (b < A.nb) A.wstart[b] = carry + (uint32_t)ex;
        carry += (uint32_t)tot;
    }
    if (threadIdx.x == 0) A.wstart[A.nb] = carry;
}

__device__ inline void put32(uint8_t *p, uint32_t v) { *reinterpret_cast<uint32_t *>(p) = v; }

// Grid: one workgroup per coding block (at least one).
__global__ void __launch_bounds__(TPC_BLOCK) rs_pack(RsBatch Bt) {
    const RsArgs A = rs_job(Bt);
    const int st0 = A.mm[2];
    const int64_t R = st0 == TPC_OK ? rs_range(A) : 0;
    const uint64_t T = st0 == TPC_OK ? (uint64_t)A.mm[3] : 0ull, T4 = (T + 3ull) & ~3ull;
    const uint64_t words = A.wstart[A.nb];
    const uint64_t head = RS_HEAD + T4 + 4ull * (A.nb + 1) + 4ull * RS_LANES * A.nb;
    const uint64_t total = head + 2ull * words;
    const bool fits = st0 == TPC_OK && total <= A.cap;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *A.out_size = st0 == TPC_OK ? total : 0ull;
        *A.dev_status = st0 != TPC_OK ? st0 : (fits ? TPC_OK : TPC_ERR_CAPACITY);
    }
    if (!fits) return;
    uint8_t *o = A.out;
    const int G = gridDim.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        put32(o, RS_MAGIC);
        put32(o + 4, 2u);
        put32(o + 8, (uint32_t)((uint64_t)A.n & 0xffffffffu));
        put32(o + 12, (uint32_t)((uint64_t)A.n >> 32));
        put32(o + 16, (uint32_t)(A.n > 0 ? A.mm[0] : 0));
        put32(o + 20, (uint32_t)R);
        put32(o + 24, (uint32_t)A.L);
        put32(o + 28, (uint32_t)A.B);
        put32(o + 32, (uint32_t)A.nb);
        put32(o + 36, (uint32_t)T);
    }
    // compressed table (zero-padded to 4 bytes), word offsets, states: spread
    // over the grid
    const uint32_t *tb = A.counts + RS_TAB_BYTES;
    uint32_t *ft = reinterpret_cast<uint32_t *>(o + RS_HEAD);
    for (int64_t q = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; q < (int64_t)(T4 / 4); q += (int64_t)G * TPC_BLOCK) {
        const uint32_t v = tb[q];
        const int64_t keep = (int64_t)T - 4 * q;                 // bytes of this word inside the table
        ft[q] = keep >= 4 ? v : (v & ((1u << (8 * keep)) - 1u));
    }
    uint32_t *ws = ft + T4 / 4;
    for (int64_t b = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; b <= A.nb; b += (int64_t)G * TPC_BLOCK) ws[b] = A.wstart[b];
    uint32_t *sts = ws + A.nb + 1;
    for (int64_t q = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; q < (int64_t)A.nb * RS_LANES; q += (int64_t)G * TPC_BLOCK)
        sts[q] = A.states[q];
    // each block's stack, last pushed first
    uint16_t *wo = reinterpret_cast<uint16_t *>(o + head);
    for (int b = blockIdx.x; b < A.nb; b += G) {
        const uint32_t top = A.wcount[b], base = A.wstart[b];
        const uint16_t *stack = A.scratch + (size_t)b * A.B;
        for (uint32_t w = threadIdx.x; w < top; w += TPC_BLOCK) wo[base + w] = stack[top - 1 - w];
    }
}

// ---------------------------------------------------------------------------
// Decoder.  rd_head parses and checks the header, rd_table builds the
// cumulative frequencies and a per-slot table (symbol, frequency, slot minus
// the symbol's cumulative start), rd_decode runs each block forwards with one
// wavefront: the lanes whose state drops below 2^16 take the next words in
// lane order (ballot rank), which is the order the encoder stored them.

struct RdArgs {
    const uint8_t *in;
    uint64_t size;
    int32_t *out;
    int64_t cap;
    int64_t *n_out;
    int32_t *dev_status;
    int64_t *hd;          // parsed header: n, lo, R, L, B, nb, word area offset, status, table bytes
    uint32_t *freq;       // [TPC_RANS_MAX_RANGE] the table, expanded
    uint32_t *vals;       // [RD_MAX_TABLE] the table's varints
    uint32_t *cum;        // [TPC_RANS_MAX_RANGE + 1]
    uint4 *slot;          // [2^16]
};

__device__ inline uint32_t get32(const uint8_t *p) { return *reinterpret_cast<const uint32_t *>(p); }

// Largest compressed table: 6 bytes for each of at most min(R, 2^16)
// present symbols.
#define RD_MAX_TABLE (6 * 65536)
__device__ inline int64_t table_bound(int64_t R) { return 6 * (R < 65536 ? R : 65536); }

__global__ void rd_head(RdArgs A) {
    if (threadIdx.x != 0) return;
    int st = TPC_OK;
    int64_t n = 0, lo = 0, R = 0, L = 0, B = 0, nb = 0, head = 0;
    int64_t T = 0;
    if (A.size < RS_HEAD || get32(A.in) != RS_MAGIC || get32(A.in + 4) != 2u) {
        st = TPC_ERR_ARG;
    } else {
        n = (int64_t)((uint64_t)get32(A.in + 8) | ((uint64_t)get32(A.in + 12) << 32));
        lo = (int32_t)get32(A.in + 16);
        R = get32(A.in + 20);
        L = get32(A.in + 24);
        B = get32(A.in + 28);
        nb = get32(A.in + 32);
        T = get32(A.in + 36);
        head = RS_HEAD + ((T + 3) & ~(int64_t)3) + 4 * (nb + 1) + 4 * (int64_t)RS_LANES * nb;
        if (n < 0 || n >= ((int64_t)1 << 31) || L < 1 || L > 16 || B < RS_LANES || B % RS_LANES ||
            R > TPC_RANS_MAX_RANGE || nb != (n > 0 ? (n + B - 1) / B : 0) || (n > 0 && R < 1) ||
            T > table_bound(R) || (uint64_t)head > A.size)
            st = TPC_ERR_ARG;
        else if (n > A.cap)
            st = TPC_ERR_CAPACITY;
    }
    int64_t *h = A.hd;
    h[0] = n; h[1] = lo; h[2] = R; h[3] = L; h[4] = B; h[5] = nb; h[6] = head; h[7] = st; h[8] = T;
}

// The table: its varints (a byte ends one when its high bit is clear; a
// varint is at most 3 bytes), then the (run, f - 1) pairs placed by a scan
// of run + 1, then the cumulative frequencies.  Malformed tables (a varint
// too long or cut off, an odd number of varints, a symbol past the range,
// f above 2^L, frequencies not summing to 2^L) are refused.
__global__ void __launch_bounds__(TPC_BLOCK) rd_table(RdArgs A) {
    __shared__ int sh[TPC_BLOCK / TPC_WAVE];
    __shared__ int bad;
    if (A.hd[7] != TPC_OK) return;
    const int64_t R = A.hd[2], L = A.hd[3], T = A.hd[8];
    const uint32_t M = 1u << L;
    const uint8_t *tb = A.in + RS_HEAD;
    if (threadIdx.x == 0) bad = 0;
    for (int64_t s = threadIdx.x; s < R; s += TPC_BLOCK) A.freq[s] = 0u;
    // varints: the one a byte ends is the number of ends before it
    int nv = 0;
    for (int64_t c0 = 0; c0 < T; c0 += TPC_BLOCK) {
        const int64_t i = c0 + threadIdx.x;
        const uint8_t bi = i < T ? tb[i] : (uint8_t)0x80;
        const int end = i < T && !(bi & 0x80);
        int tot;
        const int ex = block_exclusive_scan(end, sh, &tot);
        if (end) {
            uint32_t v = bi;
            // the continuation bytes before it (inside the table)
            int k = 1;
            while (k <= 3 && i - k >= 0 && (tb[i - k] & 0x80)) {
                v = (v << 7) | (uint32_t)(tb[i - k] & 0x7f);
                ++k;
            }
            if (k > 3) bad = 1;                               // 4 or more bytes
            A.vals[nv + ex] = v;
        }
        nv += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0 && ((T > 0 && (tb[T - 1] & 0x80)) || (nv & 1))) bad = 1;
    __threadfence_block();
    __syncthreads();
    // pairs: symbol k at (sum over pairs up to k of run + 1) - 1
    const int np = nv / 2;
    int64_t carry = 0;
    for (int c0 = 0; c0 < np && !bad; c0 += TPC_BLOCK) {
        const int k = c0 + threadIdx.x;
        uint32_t step = 0, fm1 = 0;
        if (k < np) {
            const uint32_t run = A.vals[2 * k];
            fm1 = A.vals[2 * k + 1];
            step = run < (uint32_t)R ? run + 1u : (uint32_t)R + 1u;   // past the range either way
        }
        int tot;
        const int ex = block_exclusive_scan((int)step, sh, &tot);
        if (k < np) {
            const int64_t s = carry + ex + (int64_t)step - 1;
            if (s >= R || fm1 >= M) bad = 1;
            else A.freq[s] = fm1 + 1u;
        }
        carry += tot;
        __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // 64-bit running sum: a table summing past M (however it would wrap) is refused
    uint64_t csum = 0;
    for (int64_t c0 = 0; c0 < R; c0 += TPC_BLOCK) {
        const int64_t s = c0 + threadIdx.x;
        const uint32_t v = s < R ? A.freq[s] : 0u;
        int tot;
        const int ex = block_exclusive_scan((int)v, sh, &tot);
        const uint64_t c = csum + (uint64_t)ex;
        if (s < R) A.cum[s] = c <= M ? (uint32_t)c : M;
        csum += (uint64_t)tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        A.cum[R] = csum <= M ? (uint32_t)csum : M;
        if (bad || (A.hd[0] > 0 && csum != M)) A.hd[7] = TPC_ERR_ARG;
    }
}

// Slot table: grid over symbols, each thread fills its symbol's slots.
__global__ void __launch_bounds__(TPC_BLOCK) rd_slots(RdArgs A) {
    if (A.hd[7] != TPC_OK) return;
    const int64_t R = A.hd[2];
    const uint32_t *f = A.freq;
    for (int64_t s = (int64_t)blockIdx.x * TPC_BLOCK + threadIdx.x; s < R; s += (int64_t)gridDim.x * TPC_BLOCK) {
        const uint32_t c = A.cum[s], fs = f[s];
        for (uint32_t q = 0; q < fs && c + q < (1u << 16); ++q) A.slot[c + q] = make_uint4((uint32_t)s, fs, q, 0u);
    }
}

__global__ void __launch_bounds__(TPC_BLOCK) rd_decode(RdArgs A) {
    __shared__ int failed;
    if (A.hd[7] != TPC_OK) return;                         // uniform over the grid
    const int64_t n = A.hd[0], lo = A.hd[1], R = A.hd[2], B = A.hd[4], nb = A.hd[5], head = A.hd[6];
    const int L = (int)A.hd[3];
    const uint32_t mask_M = (1u << L) - 1u;
    const uint8_t *base = A.in + RS_HEAD + ((A.hd[8] + 3) & ~(int64_t)3);
    const uint32_t *ws = reinterpret_cast<const uint32_t *>(base);
    const uint32_t *sts = ws + nb + 1;
    const uint16_t *words = reinterpret_cast<const uint16_t *>(A.in + head);
    const uint64_t n_words = (A.size - (uint64_t)head) / 2;
    const int lane = threadIdx.x & (TPC_WAVE - 1);
    if (threadIdx.x == 0) failed = 0;
    __syncthreads();
    const int64_t W = (int64_t)gridDim.x * (TPC_BLOCK / TPC_WAVE);
    for (int64_t b = (int64_t)blockIdx.x * (TPC_BLOCK / TPC_WAVE) + threadIdx.x / TPC_WAVE; b < nb; b += W) {
        const int64_t i0 = b * B, i1 = i0 + B < n ? i0 + B : n;
        uint32_t x = sts[b * RS_LANES + lane];
        uint64_t w = ws[b], w_end = ws[b + 1];
        bool ok = w <= w_end && w_end <= n_words;
        const int64_t rounds = (i1 - i0 + RS_LANES - 1) / RS_LANES;
        for (int64_t j = 0; j < rounds && ok; ++j) {
            const int64_t i = i0 + j * RS_LANES + lane;
            const bool act = i < i1;
            const uint32_t sl = x & mask_M;
            const uint4 e = act ? A.slot[sl] : make_uint4(0u, 1u, 0u, 0u);
            if (act) {
                A.out[i] = (int32_t)(lo + (int64_t)e.x);
                x = e.y * (x >> L) + e.z;
            }
            const bool need = act && x < (1u << 16);
            const unsigned long long m = __ballot(need);
            const uint32_t cnt = (uint32_t)__popcll(m);
            if (w + cnt > w_end) {
                ok = false;
                break;
            }
            if (need) {
                const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                x = (x << 16) | words[w + rank];
            }
            w += cnt;
        }
        // a block decodes back to the coders' start states, using all its words
        if (!ok || w != w_end || __ballot(x != (1u << 16)) != 0ull) failed = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && failed) A.hd[7] = TPC_ERR_ARG;
}

__global__ void rd_done(RdArgs A) {
    if (threadIdx.x == 0) {
        *A.n_out = A.hd[0];
        *A.dev_status = (int32_t)A.hd[7];
    }
}

int grid_over(int64_t items, int cap) {
    int64_t b = (items + TPC_BLOCK - 1) / TPC_BLOCK;
    if (b > cap) b = cap;
    return b < 1 ? 1 : (int)b;
}

}  // namespace

size_t rans_ws_layout(void *ws, int64_t n, int32_t B, RansWs *out) {
    WsCarver w(ws);
    const int64_t nb = n > 0 ? (n + B - 1) / B : 0;
    RansWs r;
    r.mm = w.take<int32_t>(8);
    r.counts = w.take<uint32_t>(TPC_RANS_MAX_RANGE);
    r.fc = w.take<uint4>(TPC_RANS_MAX_RANGE);
    r.wcount = w.take<uint32_t>(nb > 0 ? nb : 1);
    r.wstart = w.take<uint32_t>(nb + 1);
    r.states = w.take<uint32_t>((nb > 0 ? nb : 1) * RS_LANES);
    r.scratch = w.take<uint16_t>((size_t)(nb > 0 ? nb : 1) * B);
    if (out) *out = r;
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_rans_batch(int count, const RansJob *jobs, int32_t L, int32_t B, void *ws,
                             hipStream_t st) {
    RsBatch Bt;
    int64_t ncap = 0;
    int nb_cap = 0;
    size_t off = 0;
    for (int k = 0; k < count; ++k) {
        const RansJob &J = jobs[k];
        RansWs W;
        off += rans_ws_layout(ws ? (char *)ws + off : nullptr, J.n, B, &W);
        RsArgs &A = Bt.a[k];
        A.sym = J.sym;
        A.n = J.n;
        A.n_dev = J.n_dev;
        A.n_cap = J.n;
        A.L = L;
        A.B = B;
        A.fused = J.n >= RS_FUSE_MIN;
        A.nb = (int32_t)(J.n > 0 ? (J.n + B - 1) / B : 0);
        A.mm = W.mm;
        A.counts = W.counts;
        A.fc = W.fc;
        A.wcount = W.wcount;
        A.wstart = W.wstart;
        A.states = W.states;
        A.scratch = W.scratch;
        A.out = J.out;
        A.cap = J.cap;
        A.out_size = J.out_size;
        A.dev_status = J.dev_status;
        ncap = J.n > ncap ? J.n : ncap;
        nb_cap = A.nb > nb_cap ? A.nb : nb_cap;
    }
    // about 16 symbols per thread, at most 2048 workgroups per array
    const int gs = grid_over((ncap + 15) / 16, 2048);
    const dim3 one(1, count);
    hipLaunchKernelGGL(rs_init, one, dim3(TPC_WAVE), 0, st, Bt);
    bool any_fused = false;
    for (int k = 0; k < count; ++k) any_fused = any_fused || Bt.a[k].fused;
    if (any_fused)
        hipLaunchKernelGGL(rs_window, dim3(grid_over(TPC_RANS_MAX_RANGE, 1024), count), dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_minmax, dim3(gs, count), dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_clear, dim3(grid_over(TPC_RANS_MAX_RANGE, 1024), count), dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_hist, dim3(gs, count), dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_freq, one, dim3(RS_FREQ_THREADS), 0, st, Bt);
    hipLaunchKernelGGL(rs_table, one, dim3(TPC_BLOCK), 0, st, Bt);
    const int eb = (nb_cap + TPC_BLOCK / TPC_WAVE - 1) / (TPC_BLOCK / TPC_WAVE);
    if (eb > 0) hipLaunchKernelGGL(rs_encode, dim3(eb, count), dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_scan, one, dim3(TPC_BLOCK), 0, st, Bt);
    hipLaunchKernelGGL(rs_pack, dim3(nb_cap > 0 ? (nb_cap < 4096 ? nb_cap : 4096) : 1, count), dim3(TPC_BLOCK), 0,
                       st, Bt);
    return hipGetLastError();
}

size_t rans_batch_ws_bytes(int count, const RansJob *jobs, int32_t B) {
    size_t off = 0;
    for (int k = 0; k < count; ++k) off += rans_ws_layout(nullptr, jobs[k].n, B, nullptr);
    return off;
}

size_t rans_decode_ws_bytes() {
    WsCarver w(nullptr);
    w.take<int64_t>(9);
    w.take<uint32_t>(TPC_RANS_MAX_RANGE);
    w.take<uint32_t>(RD_MAX_TABLE);
    w.take<uint32_t>(TPC_RANS_MAX_RANGE + 1);
    w.take<uint4>(1 << 16);
    return (w.off + 255) & ~size_t(255);
}

hipError_t launch_rans_decode(const void *in, uint64_t size, int32_t *out, int64_t cap, int64_t *n_out,
                              int32_t *dev_status, void *ws, hipStream_t st) {
    RdArgs A;
    WsCarver w(ws);
    A.in = static_cast<const uint8_t *>(in);
    A.size = size;
    A.out = out;
    A.cap = cap;
    A.n_out = n_out;
    A.dev_status = dev_status;
    A.hd = w.take<int64_t>(9);
    A.freq = w.take<uint32_t>(TPC_RANS_MAX_RANGE);
    A.vals = w.take<uint32_t>(RD_MAX_TABLE);
    A.cum = w.take<uint32_t>(TPC_RANS_MAX_RANGE + 1);
    A.slot = w.take<uint4>(1 << 16);
    hipLaunchKernelGGL(rd_head, dim3(1), dim3(TPC_WAVE), 0, st, A);
    hipLaunchKernelGGL(rd_table, dim3(1), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(rd_slots, dim3(64), dim3(TPC_BLOCK), 0, st, A);
    const int64_t blocks_max = cap > 0 ? (cap + RS_LANES - 1) / RS_LANES : 1;
    int g = (int)((blocks_max + TPC_BLOCK / TPC_WAVE - 1) / (TPC_BLOCK / TPC_WAVE));
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(rd_decode, dim3(g), dim3(TPC_BLOCK), 0, st, A);
    hipLaunchKernelGGL(rd_done, dim3(1), dim3(TPC_WAVE), 0, st, A);
    return hipGetLastError();
}
