/*
 * ppc_oracle.c -- the CPU oracle for the positional population count.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.  It shares
 * no code, header, table or helper with the HIP library; the two are built
 * and loaded independently.
 *
 * What it computes is the plain definition of the operation, written out:
 *   - Fig. 2 of the paper (Section 1): for every w-bit word i and every bit
 *     position j < w, counts[j] += (word_i >> j) & 1.  Counters are added to,
 *     never cleared (Section 4, step 1 and its footnote).
 *   - Word i is the little-endian integer of bytes buf[i*s .. i*s+s-1] with
 *     s = w/8 (all machines the paper targets are little-endian; heads and
 *     tails are masked bytewise, Sections 4.1 and 4.6).
 *   - A trailing partial word is read with its missing high bytes as zero,
 *     so every byte of [buf, buf+nbytes) is counted exactly once.
 *   - Bit positions are relative to the caller's pointer, not to absolute
 *     addresses: byte buf[b] feeds counters 8*(b mod s) .. 8*(b mod s)+7.
 *
 * No SIMD, no popcount instruction, no table: one shift-and-mask per bit.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <pthread.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1

static int width_ok(unsigned w)
{
    return w == 8 || w == 16 || w == 32 || w == 64;
}

/* Fig. 2, with words assembled little-endian and a zero-padded last word. */
static void pospop_words(unsigned w, uint64_t *counts, const unsigned char *p,
                         size_t nbytes)
{
    size_t s = w / 8;
    size_t nwords = (nbytes + s - 1) / s;
    for (size_t i = 0; i < nwords; i++) {
        uint64_t word = 0;
        for (size_t b = 0; b < s; b++) {
            size_t idx = i * s + b;
            uint64_t byte = idx < nbytes ? (uint64_t)p[idx] : 0u;
            word |= byte << (8 * b);
        }
        for (unsigned j = 0; j < w; j++)
            counts[j] += (word >> j) & 1u;
    }
}

/* counts[0..w) += pospopcnt_w(buf[0..nbytes)).  Returns 0, or 1 on a bad
 * width, a NULL counts pointer, or a NULL buffer with nbytes > 0. */
int ppc_oracle_pospopcnt(unsigned w, uint64_t *counts, const void *buf,
                         size_t nbytes)
{
    if (!width_ok(w) || counts == NULL || (buf == NULL && nbytes > 0))
        return ORACLE_EINVAL;
    pospop_words(w, counts, (const unsigned char *)buf, nbytes);
    return ORACLE_OK;
}

/* ---- multithreaded wrapper, used only to time the oracle on many cores ----
 * The byte range is cut at multiples of s = w/8, so every piece starts on a
 * word boundary and its counts are plain additions to the whole (the
 * streaming use described in the footnote to Section 4, step 1). */
struct piece {
    unsigned w;
    const unsigned char *p;
    size_t n;
    uint64_t counts[64];
};

static void *piece_run(void *arg)
{
    struct piece *pc = (struct piece *)arg;
    pospop_words(pc->w, pc->counts, pc->p, pc->n);
    return NULL;
}

int ppc_oracle_pospopcnt_mt(unsigned w, uint64_t *counts, const void *buf,
                            size_t nbytes, int nthreads)
{
    if (!width_ok(w) || counts == NULL || (buf == NULL && nbytes > 0) ||
        nthreads < 1)
        return ORACLE_EINVAL;
    size_t s = w / 8;
    size_t nwords = (nbytes + s - 1) / s;
    if ((size_t)nthreads > nwords)
        nthreads = nwords > 0 ? (int)nwords : 1;
    struct piece *pcs = calloc((size_t)nthreads, sizeof *pcs);
    pthread_t *tids = calloc((size_t)nthreads, sizeof *tids);
    if (!pcs || !tids) {
        free(pcs);
        free(tids);
        return ORACLE_EINVAL;
    }
    size_t per = nwords / (size_t)nthreads, extra = nwords % (size_t)nthreads;
    size_t word0 = 0;
    for (int t = 0; t < nthreads; t++) {
        size_t nw = per + ((size_t)t < extra ? 1 : 0);
        size_t b0 = word0 * s, b1 = (word0 + nw) * s;
        if (b1 > nbytes)
            b1 = nbytes;
        pcs[t].w = w;
        pcs[t].p = (const unsigned char *)buf + b0;
        pcs[t].n = b1 > b0 ? b1 - b0 : 0;
        word0 += nw;
    }
    for (int t = 0; t < nthreads; t++) {
        if (pthread_create(&tids[t], NULL, piece_run, &pcs[t]) != 0) {
            piece_run(&pcs[t]); /* run inline if a thread cannot start */
            pcs[t].w = 0;       /* marks "not joined" */
        }
    }
    for (int t = 0; t < nthreads; t++)
        if (pcs[t].w != 0)
            pthread_join(tids[t], NULL);
    for (int t = 0; t < nthreads; t++)
        for (unsigned j = 0; j < w; j++)
            counts[j] += pcs[t].counts[j];
    free(pcs);
    free(tids);
    return ORACLE_OK;
}

/* Every (offset, length) window of one buffer, for the short/unaligned
 * sweep: out[((o * (max_len + 1)) + n) * w + j] = pospopcnt_w of
 * buf[o .. o+n) at position j, for o < n_offsets and n <= max_len.  Each
 * window is one independent evaluation of the definition above. */
int ppc_oracle_sweep(unsigned w, const void *buf, size_t max_len, size_t n_offsets,
                     uint64_t *out)
{
    if (!width_ok(w) || buf == NULL || out == NULL)
        return ORACLE_EINVAL;
    const unsigned char *p = (const unsigned char *)buf;
    for (size_t o = 0; o < n_offsets; o++)
        for (size_t n = 0; n <= max_len; n++)
            pospop_words(w, out + ((o * (max_len + 1)) + n) * w, p + o, n);
    return ORACLE_OK;
}

/* Conventional population count of a byte range (the quantity the
 * Harley-Seal algorithm of Section 3.3 computes), one bit at a time. */
uint64_t ppc_oracle_popcount(const void *buf, size_t nbytes)
{
    const unsigned char *p = (const unsigned char *)buf;
    uint64_t total = 0;
    for (size_t i = 0; i < nbytes; i++)
        for (unsigned k = 0; k < 8; k++)
            total += (p[i] >> k) & 1u;
    return total;
}
