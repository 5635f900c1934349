/*
 * CPU oracle for the entropy coder of compressed time frames: rANS over
 * arrays of 32-bit integers.  TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the CPU baseline of the benchmark call it; the GPU library never
 * does, and the two share no code.
 *
 * The paper (Sec. 4.1, compact encoding) codes every flat integer array of a time
 * frame on its own with range asymmetric numeral systems, with the symbol
 * distribution counted for each time frame, and interleaves several coders on
 * one stream.  The parameters below are this project's reading:
 *
 *   frequencies  counts c_s of the n symbols over the alphabet [lo, hi]
 *                (R = hi - lo + 1 entries, D of them present), scaled to
 *                M = 2^L:  f_s = floor(c_s (M - D) / n) + 1 for c_s > 0, else
 *                0; the shortfall M - sum f goes to the most frequent symbol
 *                (the smallest on ties).  Needs D <= M.
 *   coder        32-bit state x in [2^16, 2^32), 16-bit output words; to
 *                code s: if x >= f_s 2^(32-L), emit the low word and shift
 *                right by 16; then x <- (x div f_s) 2^L + (x mod f_s) + cum_s
 *   interleaving blocks of B symbols (B a multiple of 64); in a block, symbol
 *                j*64 + k belongs to coder k (64 coders, all starting at
 *                2^16); the block is coded backwards (j descending, k
 *                descending) onto one word stack
 *   stream       little-endian: u32 magic "RANS", u32 version 2, u64 n,
 *                i32 lo, u32 R, u32 L, u32 B, u32 number of blocks, u32 T,
 *                the frequency table in T bytes (zero-padded to a multiple
 *                of 4), u32 word_start[blocks + 1] (offsets into the word
 *                area), u32 state[blocks][64] (final coder states), u16
 *                words (each block's stack, last pushed first)
 *   table        the decoder's metadata, compressed (Sec. 4.1 says it is):
 *                for each present symbol s in ascending order, the run of
 *                absent symbols before it (s - s_prev - 1, s_prev = -1 at
 *                first) and f_s - 1, each as an unsigned LEB128 varint (7
 *                bits per byte, low group first, high bit set on every
 *                byte but the last; at most 3 bytes, as both values are
 *                below 2^21).  Absent symbols have f = 0.
 *
 * Decoding runs the block forwards (j ascending, k ascending): slot = x mod M,
 * s = the symbol with cum_s <= slot < cum_s + f_s, x <- f_s (x >> L) + slot -
 * cum_s, and if x < 2^16, x <- (x << 16) | next word.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tpc_oracle.h"

#define RANS_LANES 64
#define RANS_MAGIC 0x534E4152u     /* "RANS" */
#define RANS_LOW (1u << 16)

static void put32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t get32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

/* Scaled frequencies of counts c[0..R) with n = sum c; returns D, or -1 if
 * D > M. */
int64_t oracle_rans_freqs(const uint32_t *c, uint32_t R, uint64_t n, uint32_t L, uint32_t *f)
{
    uint64_t M = (uint64_t)1 << L;
    int64_t D = 0;
    for (uint32_t s = 0; s < R; ++s) D += c[s] > 0;
    if ((uint64_t)D > M) return -1;
    uint64_t sum = 0;
    uint32_t best = 0;
    for (uint32_t s = 0; s < R; ++s) {
        f[s] = c[s] ? (uint32_t)((uint64_t)c[s] * (M - (uint64_t)D) / n + 1) : 0;
        sum += f[s];
        if (c[s] > c[best]) best = s;
    }
    if (n) f[best] += (uint32_t)(M - sum);
    return D;
}

/* Largest table: 6 bytes for each of at most min(R, 2^16) present symbols,
 * padded to 4. */
static size_t table_bound(uint32_t R)
{
    size_t d = R < 65536u ? R : 65536u;
    return (6 * d + 3) & ~(size_t)3;
}

size_t oracle_rans_bound(int64_t n, uint32_t R, uint32_t B)
{
    uint64_t blocks = n > 0 ? ((uint64_t)n + B - 1) / B : 0;
    return 40 + table_bound(R) + 4 * (size_t)(blocks + 1) + 4 * RANS_LANES * (size_t)blocks + 2 * (size_t)n;
}

static size_t put_varint(uint8_t *p, uint32_t v)
{
    size_t k = 0;
    while (v >= 0x80u) {
        p[k++] = (uint8_t)(v | 0x80u);
        v >>= 7;
    }
    p[k++] = (uint8_t)v;
    return k;
}

/* Reads a varint of at most 3 bytes from p[*at..end); returns 0, or -1. */
static int get_varint(const uint8_t *p, size_t end, size_t *at, uint32_t *v)
{
    uint32_t x = 0;
    for (int k = 0; k < 3; ++k) {
        if (*at >= end) return -1;
        uint8_t b = p[(*at)++];
        x |= (uint32_t)(b & 0x7fu) << (7 * k);
        if (!(b & 0x80u)) { *v = x; return 0; }
    }
    return -1;
}

/* Returns 0, -1 for bad parameters or an alphabet too large, -2 if the
 * output capacity is too small (*size then holds the bound). */
int32_t oracle_rans_encode(const int32_t *sym, int64_t n, uint32_t L, uint32_t B, uint32_t max_range,
                           uint8_t *out, size_t cap, size_t *size)
{
    if (L < 1 || L > 16 || B < RANS_LANES || B % RANS_LANES || n < 0) return -1;
    int32_t lo = 0, hi = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || sym[i] < lo) lo = sym[i];
        if (i == 0 || sym[i] > hi) hi = sym[i];
    }
    uint64_t R64 = n ? (uint64_t)((int64_t)hi - (int64_t)lo) + 1 : 0;
    if (R64 > max_range) return -1;
    uint32_t R = (uint32_t)R64;
    size_t bound = oracle_rans_bound(n, R, B);
    *size = bound;
    if (cap < bound) return -2;
    uint32_t *c = (uint32_t *)calloc(R ? R : 1, 4);
    uint32_t *f = (uint32_t *)calloc(R ? R : 1, 4);
    uint32_t *cum = (uint32_t *)calloc(R ? R : 1, 4);
    for (int64_t i = 0; i < n; ++i) c[(uint32_t)((int64_t)sym[i] - lo)]++;
    if (oracle_rans_freqs(c, R, (uint64_t)n, L, f) < 0) { free(c); free(f); free(cum); return -1; }
    for (uint32_t s = 0, acc = 0; s < R; ++s) { cum[s] = acc; acc += f[s]; }
    uint32_t blocks = n ? (uint32_t)(((uint64_t)n + B - 1) / B) : 0;
    uint8_t *p = out;
    size_t T = 0;
    for (uint32_t s = 0, prev = (uint32_t)-1; s < R; ++s) {
        if (!f[s]) continue;
        T += put_varint(p + 40 + T, s - prev - 1);
        T += put_varint(p + 40 + T, f[s] - 1);
        prev = s;
    }
    put32(p, RANS_MAGIC); put32(p + 4, 2); put64(p + 8, (uint64_t)n);
    put32(p + 16, (uint32_t)lo); put32(p + 20, R); put32(p + 24, L); put32(p + 28, B);
    put32(p + 32, blocks); put32(p + 36, (uint32_t)T);
    while (T % 4) p[40 + T++] = 0;
    p += 40 + T;
    uint8_t *starts = p;
    p += 4 * (size_t)(blocks + 1);
    uint8_t *states = p;
    p += 4 * RANS_LANES * (size_t)blocks;
    uint8_t *words = p;
    uint16_t *stack = (uint16_t *)malloc(2 * (size_t)B);
    uint32_t pos = 0;
    for (uint32_t b = 0; b < blocks; ++b) {
        int64_t i0 = (int64_t)b * B, i1 = i0 + B < n ? i0 + B : n;
        uint32_t x[RANS_LANES];
        for (int k = 0; k < RANS_LANES; ++k) x[k] = RANS_LOW;
        uint32_t top = 0;
        int64_t rounds = (i1 - i0 + RANS_LANES - 1) / RANS_LANES;
        for (int64_t j = rounds - 1; j >= 0; --j) {
            for (int k = RANS_LANES - 1; k >= 0; --k) {
                int64_t i = i0 + j * RANS_LANES + k;
                if (i >= i1) continue;
                uint32_t s = (uint32_t)((int64_t)sym[i] - lo);
                uint64_t xmax = (uint64_t)f[s] << (32 - L);
                if (x[k] >= xmax) {
                    stack[top++] = (uint16_t)(x[k] & 0xFFFF);
                    x[k] >>= 16;
                }
                x[k] = ((x[k] / f[s]) << L) + (x[k] % f[s]) + cum[s];
            }
        }
        put32(starts + 4 * (size_t)b, pos);
        for (int k = 0; k < RANS_LANES; ++k) put32(states + 4 * ((size_t)b * RANS_LANES + k), x[k]);
        for (uint32_t w = 0; w < top; ++w) {          /* last pushed first */
            uint16_t v = stack[top - 1 - w];
            memcpy(words + 2 * (size_t)(pos + w), &v, 2);
        }
        pos += top;
    }
    put32(starts + 4 * (size_t)blocks, pos);
    *size = (size_t)(words - out) + 2 * (size_t)pos;
    free(stack); free(c); free(f); free(cum);
    return 0;
}

/* Returns 0, or -1 for a malformed stream or too small an output. */
int32_t oracle_rans_decode(const uint8_t *in, size_t size, int32_t *out, int64_t cap, int64_t *n_out)
{
    if (size < 40 || get32(in) != RANS_MAGIC || get32(in + 4) != 2) return -1;
    uint64_t n = get64(in + 8);
    int32_t lo = (int32_t)get32(in + 16);
    uint32_t R = get32(in + 20), L = get32(in + 24), B = get32(in + 28), blocks = get32(in + 32);
    uint32_t T = get32(in + 36);
    *n_out = (int64_t)n;
    if (L < 1 || L > 16 || B < RANS_LANES || B % RANS_LANES || (int64_t)n > cap) return -1;
    if (blocks != (n ? (uint32_t)((n + B - 1) / B) : 0) || R > (1u << 20) || T > table_bound(R)) return -1;
    size_t T4 = ((size_t)T + 3) & ~(size_t)3;
    size_t head = 40 + T4 + 4 * (size_t)(blocks + 1) + 4 * RANS_LANES * (size_t)blocks;
    if (size < head) return -1;
    const uint8_t *starts = in + 40 + T4, *states = starts + 4 * (size_t)(blocks + 1);
    const uint8_t *words = in + head;
    size_t n_words = (size - head) / 2;
    uint32_t M = 1u << L;
    uint32_t *f = (uint32_t *)malloc(4 * (size_t)(R ? R : 1));
    uint32_t *cum = (uint32_t *)malloc(4 * (size_t)(R ? R : 1));
    uint32_t *slot_sym = (uint32_t *)malloc(4 * (size_t)M);
    /* the table: (run of absent symbols, f - 1) pairs using exactly T bytes */
    int32_t bad = 0;
    memset(f, 0, 4 * (size_t)(R ? R : 1));
    for (size_t at = 40, end = 40 + (size_t)T, s = 0; at < end && !bad;) {
        uint32_t gap, fm1;
        if (get_varint(in, end, &at, &gap) || get_varint(in, end, &at, &fm1)) { bad = 1; break; }
        s += gap;
        if (s >= R || fm1 >= M) { bad = 1; break; }
        f[s++] = fm1 + 1;
    }
    uint64_t acc = 0;
    for (uint32_t s = 0; s < R; ++s) {
        cum[s] = (uint32_t)acc;
        for (uint32_t q = 0; q < f[s] && acc + q < M; ++q) slot_sym[acc + q] = s;
        acc += f[s];
    }
    int32_t st = (bad || (n && acc != M)) ? -1 : 0;
    for (uint32_t b = 0; b < blocks && !st; ++b) {
        int64_t i0 = (int64_t)b * B, i1 = i0 + B < (int64_t)n ? i0 + B : (int64_t)n;
        uint32_t x[RANS_LANES];
        for (int k = 0; k < RANS_LANES; ++k) x[k] = get32(states + 4 * ((size_t)b * RANS_LANES + k));
        size_t w = get32(starts + 4 * (size_t)b), w_end = get32(starts + 4 * (size_t)(b + 1));
        int64_t rounds = (i1 - i0 + RANS_LANES - 1) / RANS_LANES;
        for (int64_t j = 0; j < rounds && !st; ++j) {
            for (int k = 0; k < RANS_LANES; ++k) {
                int64_t i = i0 + j * RANS_LANES + k;
                if (i >= i1) continue;
                uint32_t slot = x[k] & (M - 1);
                uint32_t s = slot_sym[slot];
                out[i] = (int32_t)((int64_t)lo + s);
                x[k] = f[s] * (x[k] >> L) + slot - cum[s];
                if (x[k] < RANS_LOW) {
                    if (w >= w_end || w >= n_words) { st = -1; break; }
                    uint16_t v;
                    memcpy(&v, words + 2 * w, 2);
                    x[k] = (x[k] << 16) | v;
                    ++w;
                }
            }
        }
        /* a stream decodes back to the coders' start states */
        for (int k = 0; k < RANS_LANES && !st; ++k) if (x[k] != RANS_LOW) st = -1;
        if (!st && w != w_end) st = -1;
    }
    free(f); free(cum); free(slot_sym);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Track-model residual transform of a time frame's clusters into flat        */
/* integer arrays (the input of the entropy coder above).                     */
/*  Q(v)        rint(v * (1/q)) in single precision (1/q rounded to float),   */
/*              0 when not finite or beyond +-2^30                            */
/*  owner       a cluster belongs to the lowest-index kept track (status 0)   */
/*              holding it; clusters of no kept track are free                */
/*  per kept    seg (frame*S + sector), n (its own clusters), row0, Q(y0)     */
/*  track       and Q(z0) split as v >> 8 and v & 255, Q(y1) - Q(y0),         */
/*              Q(z1) - Q(z0) (0 where the track has fewer clusters)          */
/*  per own     for k >= 1 the row step r_k - r_(k-1) - 1; for k >= 2 the     */
/*  cluster k   second differences Q_k - 2 Q_(k-1) + Q_(k-2) in y and in z    */
/*  per segment the number of free clusters, then their Q(y), Q(z) split as   */
/*              above, in id order                                            */
/* Arrays in order: 0 trk_seg 1 trk_n 2 trk_row0 3 trk_y0h 4 trk_y0l          */
/* 5 trk_z0h 6 trk_z0l 7 trk_dy1 8 trk_dz1 9 hit_drow 10 hit_ry 11 hit_rz     */
/* 12 seg_nfree 13 free_yh 14 free_yl 15 free_zh 16 free_zl.                  */
/* ------------------------------------------------------------------------ */
static int32_t quant(float v, float inv)
{
    float s = v * inv;
    if (!(s > -1073741824.0f && s < 1073741824.0f)) return 0;
    return (int32_t)rintf(s);
}

void oracle_ctf_build(int32_t n_tracks, int32_t n_rows, int32_t n_sectors, int32_t n_segments,
                      const int32_t *row_offsets, const float *y, const float *z,
                      const int32_t *rows, const int32_t *status, const int32_t *frame,
                      const int32_t *sector, float qy, float qz, int32_t **arr, int64_t *count)
{
    int32_t N = row_offsets[n_segments];
    float iy = 1.0f / qy, iz = 1.0f / qz;
    int32_t *own = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    for (int32_t c = 0; c < N; ++c) own[c] = -1;
    for (int32_t t = n_tracks - 1; t >= 0; --t) {
        if (status[t]) continue;
        for (int32_t r = 0; r < n_rows; ++r) {
            int32_t c = rows[(size_t)t * n_rows + r];
            if (c >= 0) own[c] = t;
        }
    }
    for (int k = 0; k < 17; ++k) count[k] = 0;
    for (int32_t t = 0; t < n_tracks; ++t) {
        if (status[t]) continue;
        int32_t m = 0, r0 = 0, rp = 0, qy0 = 0, qz0 = 0, qy1 = 0, qz1 = 0, py1 = 0, pz1 = 0, py2 = 0, pz2 = 0;
        for (int32_t r = 0; r < n_rows; ++r) {
            int32_t c = rows[(size_t)t * n_rows + r];
            if (c < 0 || own[c] != t) continue;
            int32_t a = quant(y[c], iy), b = quant(z[c], iz);
            if (m == 0) { r0 = r; qy0 = a; qz0 = b; }
            else {
                arr[9][count[9]++] = r - rp - 1;
                if (m == 1) { qy1 = a; qz1 = b; }
                else {
                    arr[10][count[10]++] = a - 2 * py1 + py2;
                    arr[11][count[11]++] = b - 2 * pz1 + pz2;
                }
            }
            py2 = py1; pz2 = pz1; py1 = a; pz1 = b;
            rp = r;
            ++m;
        }
        int32_t seg = (frame[t] * n_sectors + sector[t]);
        int32_t v[9] = {seg, m, r0, qy0 >> 8, qy0 & 255, qz0 >> 8, qz0 & 255,
                        m >= 2 ? qy1 - qy0 : 0, m >= 2 ? qz1 - qz0 : 0};
        for (int k = 0; k < 9; ++k) arr[k][count[k]++] = v[k];
    }
    for (int32_t s = 0; s < n_segments; ++s) {
        int32_t nf = 0;
        for (int32_t c = row_offsets[s]; c < row_offsets[s + 1]; ++c) {
            if (own[c] >= 0) continue;
            int32_t a = quant(y[c], iy), b = quant(z[c], iz);
            arr[13][count[13]++] = a >> 8;
            arr[14][count[14]++] = a & 255;
            arr[15][count[15]++] = b >> 8;
            arr[16][count[16]++] = b & 255;
            ++nf;
        }
        arr[12][count[12]++] = nf;
    }
    free(own);
}
