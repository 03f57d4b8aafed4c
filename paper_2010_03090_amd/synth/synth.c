/*
 * Seeded synthetic inputs for UTF-8 validation: valid text with a chosen mix of
 * character lengths, uniform random bytes, single injected errors with their
 * known first-error offset, and CSR string batches.
 *
 * This module only *writes* UTF-8 (it encodes code points); it holds none of
 * the validation arithmetic.  Every output is a pure function of the seed and
 * the arguments, independent of the number of threads.
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based
 * generator: stream s draws splitmix64(seed_s + k * 0x9E3779B97F4A7C15).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } rng_t;

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static uint64_t rng_next(rng_t *r) { r->s += 0x9E3779B97F4A7C15ULL; return mix64(r->s); }
static rng_t rng_stream(uint64_t seed, uint64_t stream) { rng_t r = { mix64(seed ^ mix64(stream + 0x632BE59BD9B4E019ULL)) }; return r; }
static uint64_t rng_below(rng_t *r, uint64_t n) { return n ? rng_next(r) % n : 0; }   /* bias < 2^-40 for our n */
static double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* ---- character classes: byte length 1..4 ---------------------------------- */

/* Draw a code point whose UTF-8 form has exactly `len` bytes (surrogates excluded). */
static uint32_t draw_cp(rng_t *r, int len)
{
    switch (len) {
    case 1: return (uint32_t)rng_below(r, 0x80);
    case 2: return 0x80 + (uint32_t)rng_below(r, 0x800 - 0x80);
    case 3: {
        /* 0x800..0xFFFF minus 0xD800..0xDFFF: 61440 values */
        uint32_t v = 0x800 + (uint32_t)rng_below(r, 0x10000 - 0x800 - 0x800);
        return v >= 0xD800 ? v + 0x800 : v;
    }
    default: return 0x10000 + (uint32_t)rng_below(r, 0x110000 - 0x10000);
    }
}

static int encode_cp(uint32_t cp, uint8_t *o)
{
    if (cp < 0x80) { o[0] = (uint8_t)cp; return 1; }
    if (cp < 0x800) { o[0] = (uint8_t)(0xC0 | (cp >> 6)); o[1] = (uint8_t)(0x80 | (cp & 0x3F)); return 2; }
    if (cp < 0x10000) {
        o[0] = (uint8_t)(0xE0 | (cp >> 12)); o[1] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
        o[2] = (uint8_t)(0x80 | (cp & 0x3F)); return 3;
    }
    o[0] = (uint8_t)(0xF0 | (cp >> 18)); o[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
    o[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F)); o[3] = (uint8_t)(0x80 | (cp & 0x3F)); return 4;
}

/* Probability (in 1/2^16 units, cumulative) of byte lengths 1..4 per variant. */
enum { V_ASCII = 0, V_LATIN, V_CJK, V_EMOJI, V_RANDOM, V_MIXED, V_UNIF1, V_UNIF2, V_UNIF3, V_UNIF4, V_COUNT };

static const uint32_t k_cum[V_COUNT][4] = {
    /* ASCII   */ { 65536, 65536, 65536, 65536 },
    /* Latin   */ { 55706, 65536, 65536, 65536 },          /* 85% / 15% */
    /* CJK     */ { 6554, 6554, 65536, 65536 },            /* 10% 1-byte / 90% 3-byte */
    /* emoji   */ { 26214, 26214, 26214, 65536 },          /* 40% / 60% 4-byte */
    /* random  */ { 0, 0, 0, 0 },                          /* uniform bytes, handled apart */
    /* mixed   */ { 32768, 45875, 58982, 65536 },          /* 50 / 20 / 20 / 10 */
    /* paper's generator: byte length uniform over {1}, {1,2}, {1,2,3}, {1,2,3,4} */
    { 65536, 65536, 65536, 65536 },
    { 32768, 65536, 65536, 65536 },
    { 21845, 43691, 65536, 65536 },
    { 16384, 32768, 49152, 65536 },
};

static int draw_len(rng_t *r, int variant, int max_len)
{
    const uint32_t *c = k_cum[variant];
    if (max_len >= 4) {
        uint32_t u = (uint32_t)(rng_next(r) >> 48);
        int len = 1;
        while (len < 4 && u >= c[len - 1]) len++;
        return len;
    }
    /* The last characters are restricted to lengths that still fit: draw with
     * the variant's weights renormalised over lengths 1..max_len (ASCII when
     * none of them has weight). */
    uint32_t total = c[max_len - 1];
    if (total == 0) return 1;
    uint32_t v = (uint32_t)rng_below(r, total);
    int len = 1;
    while (len < max_len && v >= c[len - 1]) len++;
    return len;
}

/* Fill out[0..n) with valid text of the variant; exact length. */
static void fill_text(uint8_t *out, int64_t n, int variant, rng_t *r)
{
    if (variant == V_RANDOM) {
        int64_t i = 0;
        for (; i + 8 <= n; i += 8) { uint64_t v = rng_next(r); memcpy(out + i, &v, 8); }
        if (i < n) { uint64_t v = rng_next(r); memcpy(out + i, &v, (size_t)(n - i)); }
        return;
    }
    int64_t i = 0;
    uint8_t tmp[4];
    while (i < n) {
        int64_t left = n - i;
        int len = draw_len(r, variant, left < 4 ? (int)left : 4);
        int w = encode_cp(draw_cp(r, len), tmp);
        memcpy(out + i, tmp, (size_t)w);
        i += w;
    }
}

#define CHUNK ((int64_t)1 << 20)

struct text_job { uint8_t *out; int64_t n; int variant; uint64_t seed; int64_t c0, c1; };

static void *text_worker(void *arg)
{
    struct text_job *j = (struct text_job *)arg;
    for (int64_t c = j->c0; c < j->c1; c++) {
        int64_t b = c * CHUNK, e = b + CHUNK < j->n ? b + CHUNK : j->n;
        rng_t r = rng_stream(j->seed, (uint64_t)c);
        fill_text(j->out + b, e - b, j->variant, &r);
    }
    return NULL;
}

/* Valid text (or random bytes) of exactly n bytes; 1 MiB chunks are independent streams. */
int synth_text(uint8_t *out, int64_t n, int variant, uint64_t seed, int nthreads)
{
    if (n < 0 || variant < 0 || variant >= V_COUNT) return -1;
    int64_t chunks = (n + CHUNK - 1) / CHUNK;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (chunks < nthreads) nthreads = chunks > 0 ? (int)chunks : 1;
    pthread_t tid[64];
    struct text_job jobs[64];
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (struct text_job){ out, n, variant, seed, chunks * t / nthreads, chunks * (t + 1) / nthreads };
    }
    if (nthreads == 1) { text_worker(&jobs[0]); return 0; }
    for (int t = 0; t < nthreads; t++) pthread_create(&tid[t], NULL, text_worker, &jobs[t]);
    for (int t = 0; t < nthreads; t++) pthread_join(tid[t], NULL);
    return 0;
}

/* ---- error injection ---------------------------------------------------------- */

enum { E_LONE_CONT = 0, E_TRUNCATED, E_OVERLONG, E_TOO_LARGE, E_SURROGATE, E_FIVE_PLUS, E_CUT_AT_END, E_COUNT };

static uint8_t cont(rng_t *r, uint8_t lo, uint8_t hi) { return (uint8_t)(lo + rng_below(r, (uint64_t)(hi - lo) + 1)); }
static int is_cont(uint8_t b) { return (b & 0xC0) == 0x80; }

/* Error pattern of a class that fits in `room` bytes (room >= 1); returns its length, 0 if none fits. */
static int make_pattern(int cls, int room, rng_t *r, uint8_t *p)
{
    switch (cls) {
    case E_LONE_CONT:
        p[0] = cont(r, 0x80, 0xBF); return 1;
    case E_TRUNCATED: {
        /* lead of an L-byte character keeping 1..L-1 of its bytes, then an ASCII byte */
        int L = 2 + (int)rng_below(r, 3);
        int keep = 1 + (int)rng_below(r, (uint64_t)(L - 1));
        if (keep + 1 > room) { L = 2; keep = 1; if (room < 2) return 0; }
        uint8_t tmp[4];
        encode_cp(draw_cp(r, L), tmp);
        memcpy(p, tmp, (size_t)keep);
        p[keep] = (uint8_t)(0x20 + rng_below(r, 0x5F));
        return keep + 1;
    }
    case E_OVERLONG: {
        int k = (int)rng_below(r, 3);
        if (k == 2 && room < 4) k = room >= 3 ? 1 : 0;
        if (k == 1 && room < 3) k = 0;
        if (room < 2) return 0;
        if (k == 0) { p[0] = (uint8_t)(0xC0 + rng_below(r, 2)); p[1] = cont(r, 0x80, 0xBF); return 2; }
        if (k == 1) { p[0] = 0xE0; p[1] = cont(r, 0x80, 0x9F); p[2] = cont(r, 0x80, 0xBF); return 3; }
        p[0] = 0xF0; p[1] = cont(r, 0x80, 0x8F); p[2] = cont(r, 0x80, 0xBF); p[3] = cont(r, 0x80, 0xBF); return 4;
    }
    case E_TOO_LARGE: {
        /* four-byte form of U+110000..1FFFFF */
        if (room < 4) return 0;
        uint32_t cp = 0x110000 + (uint32_t)rng_below(r, 0x200000 - 0x110000);
        p[0] = (uint8_t)(0xF0 | (cp >> 18)); p[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
        p[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F)); p[3] = (uint8_t)(0x80 | (cp & 0x3F));
        return 4;
    }
    case E_SURROGATE:
        if (room < 3) return 0;
        p[0] = 0xED; p[1] = cont(r, 0xA0, 0xBF); p[2] = cont(r, 0x80, 0xBF); return 3;
    case E_FIVE_PLUS: {
        int m = room < 4 ? room : 4;
        p[0] = (uint8_t)(0xF5 + rng_below(r, 11));
        for (int k = 1; k < m; k++) p[k] = cont(r, 0x80, 0xBF);
        return m;
    }
    default: return 0;
    }
}

/*
 * Inject one error into valid text buf[0..n) at the first character boundary at
 * or after `pos` (class `cls`).  The characters covering the pattern are
 * replaced by it and padded with ASCII, so the length is unchanged and the
 * text after them is untouched.  E_CUT_AT_END truncates the last character
 * instead.  Returns the expected first-error offset, or -1 if it did not fit.
 */
int64_t synth_inject(uint8_t *buf, int64_t n, int64_t pos, int cls, uint64_t seed)
{
    if (n <= 0 || cls < 0 || cls >= E_COUNT) return -1;
    rng_t r = rng_stream(seed, 0xE77);
    if (pos < 0) pos = 0;
    if (pos >= n) pos = n - 1;
    if (cls == E_CUT_AT_END) {
        /* the text ends inside a character: rewrite the last character as the
         * first (room) bytes of a longer one */
        int64_t s = n - 1;
        while (s > 0 && is_cont(buf[s])) s--;
        int64_t room = n - s;                     /* 1..4 */
        if (room >= 4) { buf[s] = (uint8_t)('a' + rng_below(&r, 26)); s++; room = n - s; }
        int L = (int)room + 1 + (int)rng_below(&r, (uint64_t)(4 - room));
        uint8_t tmp[4];
        encode_cp(draw_cp(&r, L), tmp);
        memcpy(buf + s, tmp, (size_t)room);
        return s;
    }
    int64_t s = pos;
    while (s < n && is_cont(buf[s])) s++;
    if (s >= n) return -1;
    uint8_t p[8];
    int m = make_pattern(cls, (int)(n - s < 8 ? n - s : 8), &r, p);
    if (m == 0) return -1;
    /* cover whole characters starting at s */
    int64_t e = s;
    while (e < s + m) { e++; while (e < n && is_cont(buf[e])) e++; }
    if (e > n) return -1;
    memcpy(buf + s, p, (size_t)m);
    for (int64_t k = s + m; k < e; k++) buf[k] = (uint8_t)('a' + rng_below(&r, 26));
    return s;
}

/* ---- CSR batches --------------------------------------------------------------- */

enum { L_LOGNORMAL = 0, L_PARETO = 1 };

/* Draw n string lengths. LOGNORMAL: round(exp(ln(a) + b z)) clipped to [lo, hi].
 * PARETO: floor(a / u^(1/b)) clipped to [lo, hi]. */
int synth_lengths(int64_t *len, int64_t n, int dist, double a, double b, int64_t lo, int64_t hi, uint64_t seed)
{
    if (n < 0) return -1;
    rng_t r = rng_stream(seed, 0x1E6);
    for (int64_t k = 0; k < n; k++) {
        double v;
        if (dist == L_LOGNORMAL) {
            double u1 = rng_unit(&r), u2 = rng_unit(&r);
            if (u1 < 1e-300) u1 = 1e-300;
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            v = floor(exp(log(a) + b * z) + 0.5);
        } else {
            double u = 1.0 - rng_unit(&r);
            v = floor(a / pow(u, 1.0 / b));
        }
        if (!(v >= (double)lo)) v = (double)lo;
        if (v > (double)hi) v = (double)hi;
        len[k] = (int64_t)v;
    }
    return 0;
}

struct batch_job {
    uint8_t *data; const int64_t *offsets; const int32_t *variant; int64_t k0, k1; uint64_t seed;
};

static void *batch_worker(void *arg)
{
    struct batch_job *j = (struct batch_job *)arg;
    for (int64_t k = j->k0; k < j->k1; k++) {
        rng_t r = rng_stream(j->seed, (uint64_t)k);
        fill_text(j->data + j->offsets[k], j->offsets[k + 1] - j->offsets[k], j->variant[k], &r);
    }
    return NULL;
}

/* Fill each string k = data[offsets[k]..offsets[k+1]) with valid text of variant[k]. */
int synth_batch_text(uint8_t *data, const int64_t *offsets, const int32_t *variant, int64_t n,
                     uint64_t seed, int nthreads)
{
    if (n < 0) return -1;
    for (int64_t k = 0; k < n; k++)
        if (variant[k] < 0 || variant[k] >= V_COUNT) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    if (n < nthreads * 16) nthreads = 1;
    pthread_t tid[64];
    struct batch_job jobs[64];
    for (int t = 0; t < nthreads; t++)
        jobs[t] = (struct batch_job){ data, offsets, variant, n * t / nthreads, n * (t + 1) / nthreads, seed };
    if (nthreads == 1) { batch_worker(&jobs[0]); return 0; }
    for (int t = 0; t < nthreads; t++) pthread_create(&tid[t], NULL, batch_worker, &jobs[t]);
    for (int t = 0; t < nthreads; t++) pthread_join(tid[t], NULL);
    return 0;
}
