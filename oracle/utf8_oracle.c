/*
 * UTF-8 validation oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant with the GPU
 * validator: it is the plain definition the GPU result is checked against.
 *
 * Definition followed (Keiser & Lemire, "Validating UTF-8 In Less Than One
 * Instruction Per Byte"):
 *   - Table 1 (section 2) gives the byte ranges of every well-formed character
 *     (RFC 3629): one byte 00..7F; two bytes C2..DF + 80..BF; three bytes
 *     E0 A0..BF 80..BF, E1..EC/EE..EF 80..BF 80..BF, ED 80..9F 80..BF; four
 *     bytes F0 90..BF, F1..F3 80..BF, F4 80..8F, each followed by two 80..BF.
 *   - Section 3 lists the six rules (5+ byte, too short, too long, overlong,
 *     too large, surrogate) that any byte outside those ranges violates.
 *   - Algorithm 1 (section 4) is the branchy range walk used here: switch on
 *     the lead byte, then check the count and range of continuation bytes.
 *     Its four-byte case led by F4 is read with the continuation range 80..8F
 *     (Table 4 lists F4 90 80 80 as too large, and Table 1 ends at F4 8F BF BF);
 *     the printed listing only excludes A0..BF there.
 *
 * Result convention (the paper only decides a boolean): the first-error offset
 * of a byte string is the length of its longest valid prefix made of whole
 * characters, i.e. the start of the first ill-formed character met by a
 * left-to-right walk, or -1 when the whole string is valid.  The empty string
 * is valid.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* Continuation byte check: a byte of the form 10xxxxxx (section 2). */
static int in_range(uint8_t c, uint8_t lo, uint8_t hi) { return c >= lo && c <= hi; }

/*
 * Length of the well-formed character starting at b[i], or 0 if the bytes at
 * b[i..] do not begin a well-formed character (Algorithm 1 with the F4 fix).
 */
static int char_len(const uint8_t *b, int64_t i, int64_t n)
{
    uint8_t c = b[i];
    int len;
    uint8_t lo1 = 0x80, hi1 = 0xBF; /* allowed range of the first continuation */
    if (c <= 0x7F) return 1;                         /* ASCII, U+0000..007F */
    else if (in_range(c, 0xC2, 0xDF)) len = 2;       /* U+0080..07FF */
    else if (c == 0xE0) { len = 3; lo1 = 0xA0; }     /* U+0800..0FFF: 80..9F would be overlong */
    else if (c == 0xED) { len = 3; hi1 = 0x9F; }     /* U+D000..D7FF: A0..BF would be surrogates */
    else if (in_range(c, 0xE1, 0xEC) || in_range(c, 0xEE, 0xEF)) len = 3;
    else if (c == 0xF0) { len = 4; lo1 = 0x90; }     /* U+10000..3FFFF: 80..8F would be overlong */
    else if (in_range(c, 0xF1, 0xF3)) len = 4;       /* U+40000..FFFFF */
    else if (c == 0xF4) { len = 4; hi1 = 0x8F; }     /* U+100000..10FFFF: 90..BF too large */
    else return 0;  /* 80..BF too long (stray continuation), C0/C1 overlong, F5..FF too large / 5+ bytes */

    if (i + len > n) return 0;                       /* too short: input ends inside the character */
    if (!in_range(b[i + 1], lo1, hi1)) return 0;
    for (int k = 2; k < len; k++)
        if (!in_range(b[i + k], 0x80, 0xBF)) return 0;
    return len;
}

/* First-error offset of b[0..n): -1 if valid. */
int64_t oracle_first_error(const uint8_t *b, int64_t n)
{
    int64_t i = 0;
    while (i < n) {
        int len = char_len(b, i, n);
        if (len == 0) return i;
        i += len;
    }
    return -1;
}

/* Per-string results for a CSR batch: string k is data[offsets[k] .. offsets[k+1]). */
struct batch_job {
    const uint8_t *data;
    const int64_t *offsets;
    int64_t begin, end;
    uint8_t *flags;
    int64_t *first_err;
};

static void *batch_worker(void *arg)
{
    struct batch_job *j = (struct batch_job *)arg;
    for (int64_t k = j->begin; k < j->end; k++) {
        int64_t s = j->offsets[k], e = j->offsets[k + 1];
        int64_t r = oracle_first_error(j->data + s, e - s);
        j->first_err[k] = r;
        j->flags[k] = (uint8_t)(r < 0);
    }
    return NULL;
}

/* Offsets are relative to each string's start; runs on nthreads host threads. */
int oracle_first_error_batch(const uint8_t *data, const int64_t *offsets, int64_t n,
                             uint8_t *flags, int64_t *first_err, int nthreads)
{
    if (n < 0 || nthreads < 1) return -1;
    if (nthreads > 256) nthreads = 256;
    if (n < (int64_t)nthreads * 64) nthreads = 1;
    pthread_t tid[256];
    struct batch_job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].data = data; jobs[t].offsets = offsets;
        jobs[t].begin = n * t / nthreads; jobs[t].end = n * (t + 1) / nthreads;
        jobs[t].flags = flags; jobs[t].first_err = first_err;
    }
    if (nthreads == 1) { batch_worker(&jobs[0]); return 0; }
    for (int t = 0; t < nthreads; t++)
        if (pthread_create(&tid[t], NULL, batch_worker, &jobs[t]) != 0) {
            for (int u = 0; u < t; u++) pthread_join(tid[u], NULL);
            return -2;
        }
    for (int t = 0; t < nthreads; t++) pthread_join(tid[t], NULL);
    return 0;
}

/*
 * Error class of the ill-formed character starting at b[s] (s = a first-error
 * offset, 0 <= s < n), by the six rules of section 3, taken in this order:
 *   1  a) 5+ byte   -- the lead byte has five or more header bits (F8..FF);
 *   3  c) too long  -- the lead byte is a continuation byte (80..BF);
 *   2  b) too short -- the lead's header bits announce N bytes (C0..DF: 2,
 *                      E0..EF: 3, F0..F7: 4) but fewer than N-1 continuation
 *                      bytes follow before another byte or the end;
 * and, for a well-formed sequence, on its decoded code point:
 *   4  d) overlong  -- below the smallest value of its length (80, 800, 10000);
 *   5  e) too large -- above U+10FFFF;
 *   6  f) surrogate -- in U+D800..DFFF.
 * The malformed rules come first because only a well-formed sequence decodes to
 * a code point.  Returns 0 if s is out of range or the character is valid.
 * Codes: 1..6 = rules a..f.
 */
int oracle_error_class(const uint8_t *b, int64_t n, int64_t s)
{
    if (s < 0 || s >= n) return 0;
    uint8_t c = b[s];
    if (c >= 0xF8) return 1;                                   /* a) five or more header bits */
    if (c >= 0x80 && c <= 0xBF) return 3;                      /* c) continuation as lead */
    if (c <= 0x7F) return 0;                                   /* ASCII is always valid */
    int len = c >= 0xF0 ? 4 : c >= 0xE0 ? 3 : 2;
    for (int k = 1; k < len; k++)
        if (s + k >= n || !in_range(b[s + k], 0x80, 0xBF)) return 2;   /* b) too short */
    uint32_t cp = (uint32_t)(c & (0x7F >> len));               /* payload bits of the lead */
    for (int k = 1; k < len; k++) cp = (cp << 6) | (b[s + k] & 0x3F);
    static const uint32_t min_cp[5] = {0, 0, 0x80, 0x800, 0x10000};
    if (cp < min_cp[len]) return 4;                            /* d) overlong */
    if (cp > 0x10FFFF) return 5;                               /* e) too large */
    if (cp >= 0xD800 && cp <= 0xDFFF) return 6;                /* f) surrogate */
    return 0;
}

/* Error class per string of a CSR batch, from its first-error offset (0 for valid strings). */
int oracle_error_class_batch(const uint8_t *data, const int64_t *offsets, int64_t n, const int64_t *first_err,
                             uint8_t *out)
{
    if (n < 0) return -1;
    for (int64_t k = 0; k < n; k++) {
        int64_t st = offsets[k], len = offsets[k + 1] - st;
        out[k] = (uint8_t)(first_err[k] < 0 ? 0 : oracle_error_class(data + st, len, first_err[k]));
    }
    return 0;
}

/*
 * Brute force over every byte string of length len (len <= 4): hist[k] counts
 * the strings whose first-error offset is k (0 <= k < len) and hist[len] counts
 * the valid ones.
 */
int oracle_exhaustive_hist(int len, uint64_t *hist)
{
    if (len < 0 || len > 4) return -1;
    for (int k = 0; k <= len; k++) hist[k] = 0;
    uint64_t total = 1;
    for (int k = 0; k < len; k++) total *= 256;
    uint8_t b[4];
    for (uint64_t v = 0; v < total; v++) {
        uint64_t w = v;
        for (int k = 0; k < len; k++) { b[k] = (uint8_t)(w & 0xFF); w >>= 8; }
        int64_t r = oracle_first_error(b, len);
        hist[r < 0 ? len : r]++;
    }
    return 0;
}
