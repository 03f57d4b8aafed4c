/*
 * Host CPU baseline: the lookup algorithm of section 6 with AVX2, as the paper
 * runs it, for throughput comparisons only.  The library never calls this code
 * (there is no CPU path in the product); bench.py times it next to the GPU.
 *
 * Per 32-byte register (section 6): prev1..prev3 come from the previous
 * register by byte alignment; three 16-entry nibble tables are looked up with
 * vpshufb (high nibble of prev1, low nibble of prev1, high nibble of the byte)
 * and ANDed (section 6.1, tables in the bit order of Table 9); the bytes that
 * must be second/third continuations (prev2 >= E0 or prev3 >= F0, section 6.2)
 * are XORed with bit 7; 64-byte blocks that are all ASCII only check that the
 * previous block did not end inside a character (section 6.4); the end of the
 * input must not cut a character (section 6.3).  Validity only (a boolean).
 */
#include <immintrin.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

__attribute__((target("avx2"))) static inline __m256i prev_n(__m256i cur, __m256i prev, int n) {
    /* bytes [i-n] of the 64-byte stream prev:cur, for the 32 positions of cur */
    __m256i t = _mm256_permute2x128_si256(prev, cur, 0x21);  /* prev.hi : cur.lo */
    switch (n) {
    case 1: return _mm256_alignr_epi8(cur, t, 15);
    case 2: return _mm256_alignr_epi8(cur, t, 14);
    default: return _mm256_alignr_epi8(cur, t, 13);
    }
}

struct state {
    __m256i prev, err, incomplete;
};

__attribute__((target("avx2"))) static void step(struct state *s, __m256i in) {
    const __m256i t1 = _mm256_setr_epi8(0x02, 0x02, 0x02, 0x02, 0x02, 0x02, 0x02, 0x02, (char)0x80, (char)0x80,
                                        (char)0x80, (char)0x80, 0x21, 0x01, 0x15, 0x49, 0x02, 0x02, 0x02, 0x02, 0x02,
                                        0x02, 0x02, 0x02, (char)0x80, (char)0x80, (char)0x80, (char)0x80, 0x21, 0x01,
                                        0x15, 0x49);
    const __m256i t2 = _mm256_setr_epi8(
        (char)0xE7, (char)0xA3, (char)0x83, (char)0x83, (char)0x8B, (char)0xCB, (char)0xCB, (char)0xCB, (char)0xCB,
        (char)0xCB, (char)0xCB, (char)0xCB, (char)0xCB, (char)0xDB, (char)0xCB, (char)0xCB, (char)0xE7, (char)0xA3,
        (char)0x83, (char)0x83, (char)0x8B, (char)0xCB, (char)0xCB, (char)0xCB, (char)0xCB, (char)0xCB, (char)0xCB,
        (char)0xCB, (char)0xCB, (char)0xDB, (char)0xCB, (char)0xCB);
    const __m256i t3 = _mm256_setr_epi8(0x01, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01, (char)0xE6, (char)0xAE,
                                        (char)0xBA, (char)0xBA, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01, 0x01,
                                        0x01, 0x01, 0x01, (char)0xE6, (char)0xAE, (char)0xBA, (char)0xBA, 0x01, 0x01,
                                        0x01, 0x01);
    const __m256i lo4 = _mm256_set1_epi8(0x0F);
    const __m256i p1 = prev_n(in, s->prev, 1);
    const __m256i h1 = _mm256_and_si256(_mm256_srli_epi16(p1, 4), lo4);
    const __m256i l1 = _mm256_and_si256(p1, lo4);
    const __m256i h2 = _mm256_and_si256(_mm256_srli_epi16(in, 4), lo4);
    const __m256i sc = _mm256_and_si256(_mm256_and_si256(_mm256_shuffle_epi8(t1, h1), _mm256_shuffle_epi8(t2, l1)),
                                        _mm256_shuffle_epi8(t3, h2));
    /* second / third continuation required: prev2 >= E0 or prev3 >= F0 (saturating subtract leaves bit 7) */
    const __m256i p2 = prev_n(in, s->prev, 2);
    const __m256i p3 = prev_n(in, s->prev, 3);
    const __m256i need = _mm256_or_si256(_mm256_subs_epu8(p2, _mm256_set1_epi8((char)(0xE0 - 0x80))),
                                         _mm256_subs_epu8(p3, _mm256_set1_epi8((char)(0xF0 - 0x80))));
    const __m256i m23 = _mm256_and_si256(need, _mm256_set1_epi8((char)0x80));
    s->err = _mm256_or_si256(s->err, _mm256_xor_si256(m23, sc));
    /* a character still open at the end of this register */
    const __m256i maxv = _mm256_setr_epi8(-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                          -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, (char)(0xF0 - 1), (char)(0xE0 - 1),
                                          (char)(0xC0 - 1));
    s->incomplete = _mm256_subs_epu8(in, maxv);
    s->prev = in;
}

/* 1 if buf[0..n) is valid UTF-8; `before` (may be NULL) holds the 32 bytes preceding buf. */
__attribute__((target("avx2"))) static int validate_span(const uint8_t *buf, int64_t n, const uint8_t *before,
                                                         int end_check) {
    struct state s;
    s.prev = before ? _mm256_loadu_si256((const __m256i *)before) : _mm256_setzero_si256();
    s.err = _mm256_setzero_si256();
    s.incomplete = _mm256_setzero_si256();
    if (before) {
        const __m256i maxv = _mm256_setr_epi8(-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1,
                                              -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, (char)(0xF0 - 1),
                                              (char)(0xE0 - 1), (char)(0xC0 - 1));
        s.incomplete = _mm256_subs_epu8(s.prev, maxv);
    }
    int64_t i = 0;
    for (; i + 64 <= n; i += 64) {
        const __m256i a = _mm256_loadu_si256((const __m256i *)(buf + i));
        const __m256i b = _mm256_loadu_si256((const __m256i *)(buf + i + 32));
        if (_mm256_movemask_epi8(_mm256_or_si256(a, b)) == 0) {   /* all ASCII (section 6.4) */
            s.err = _mm256_or_si256(s.err, s.incomplete);
            s.prev = b;
            s.incomplete = _mm256_setzero_si256();
            continue;
        }
        step(&s, a);
        step(&s, b);
    }
    if (i < n) {  /* the tail, padded with zeros */
        uint8_t pad[64];
        memset(pad, 0, sizeof pad);
        memcpy(pad, buf + i, (size_t)(n - i));
        step(&s, _mm256_loadu_si256((const __m256i *)pad));
        if (n - i > 32) step(&s, _mm256_loadu_si256((const __m256i *)(pad + 32)));
        /* the zero padding acts as the end: its first byte carries the end check */
    }
    /* the end must not cut a character (a span that is not the end has a length of a multiple of 64) */
    if (end_check) s.err = _mm256_or_si256(s.err, s.incomplete);
    return _mm256_testz_si256(s.err, s.err);
}

int host_lookup_supported(void) { return __builtin_cpu_supports("avx2") ? 1 : 0; }

/* 1 valid, 0 invalid, -1 no AVX2. */
int host_lookup_validate(const uint8_t *buf, int64_t n) {
    if (!host_lookup_supported()) return -1;
    return validate_span(buf, n, NULL, 1);
}

struct job {
    const uint8_t *buf;
    int64_t a, b, n;
    int ok;
};

static void *worker(void *p) {
    struct job *j = (struct job *)p;
    /* every span but the first starts at least 1 MiB in, so 32 bytes precede it */
    j->ok = validate_span(j->buf + j->a, j->b - j->a, j->a ? j->buf + j->a - 32 : NULL, j->b == j->n);
    return NULL;
}

/* Multi-threaded: contiguous spans of a multiple of 64 bytes; each starts from the 32 bytes before it. */
int host_lookup_validate_mt(const uint8_t *buf, int64_t n, int nthreads) {
    if (!host_lookup_supported()) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    int64_t per = (n / nthreads) & ~(int64_t)63;
    if (per < (1 << 20)) return validate_span(buf, n, NULL, 1);
    pthread_t tid[256];
    struct job jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].buf = buf;
        jobs[t].n = n;
        jobs[t].a = per * t;
        jobs[t].b = t == nthreads - 1 ? n : per * (t + 1);
        pthread_create(&tid[t], NULL, worker, &jobs[t]);
    }
    int ok = 1;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(tid[t], NULL);
        ok &= jobs[t].ok;
    }
    return ok;
}
