/*
 * ppc.h -- positional population count (pospopcnt) on AMD Instinct MI355X.
 *
 * The operation (Clausecker, Lemire, Schintke, "Faster Positional-Population
 * Counts for AVX2, AVX-512, and ASIMD", Section 1, Fig. 2): for an array of
 * w-bit words, counts[j] += number of words whose bit j is set, j < w,
 * w in {8, 16, 32, 64}.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory.  `buf` and `counts` are DEVICE pointers (memory of the current
 *    HIP device).  The caller owns both.  `counts` holds w uint64 values and
 *    must be 8-byte aligned.  `buf` may have any byte alignment.
 *  - Words.  Word i is the little-endian integer of bytes buf[i*s .. i*s+s-1],
 *    s = w/8.  Bit positions are relative to `buf`, not to absolute
 *    addresses: byte buf[b] feeds counters 8*(b mod s) .. 8*(b mod s)+7.
 *    A trailing partial word is counted as if zero-padded; `nbytes` may be
 *    any value.  Bytes outside [buf, buf+nbytes) are never read.
 *  - Accumulation.  Counts are ADDED to `counts`, never cleared (Section 4,
 *    step 1 and its footnote: this is what streamed input needs).  Counters
 *    wrap modulo 2^64.
 *  - Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Every call only enqueues work and returns; results are valid
 *    once the stream has reached that point.
 *  - Errors.  Every call returns a ppc_status.  Invalid arguments return
 *    PPC_EINVAL and enqueue nothing; a failed HIP call returns PPC_EDEVICE.
 *    No call aborts the process.  nbytes == 0 is a successful no-op (buf may
 *    then be NULL).
 *  - Aliasing.  `counts` must not overlap `buf`.
 */
#ifndef PPC_H
#define PPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ppc_status {
    PPC_OK = 0,      /* success                                            */
    PPC_EINVAL = 1,  /* invalid argument (bad width, NULL, misaligned ...)  */
    PPC_ENOMEM = 2,  /* a host or device allocation failed                 */
    PPC_EDEVICE = 3, /* a HIP runtime call or kernel launch failed         */
    PPC_EBUSY = 4    /* not admitted now (serving); retry later            */
} ppc_status;

/* Human-readable name of a status code.  Never NULL. */
const char *ppc_status_string(int status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int ppc_version(void);

/* ------------------------------------------------------------------------
 * Plain calls, one per width (Section 4; the width only changes the final
 * accumulation function f_w, Section 5).  counts[0..w) += pospopcnt_w of
 * buf[0..nbytes).  The kernel counts 64 bit positions relative to absolute
 * addresses mod 8 and then folds them to w positions relative to `buf`.
 * No scratch memory: per-block partial counts live in LDS and are added to
 * `counts` with 64-bit device atomics (order-independent, so exact).
 * ---------------------------------------------------------------------- */
ppc_status ppc_pospopcnt8(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt16(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt32(uint64_t *counts, const void *buf, size_t nbytes, void *stream);
ppc_status ppc_pospopcnt64(uint64_t *counts, const void *buf, size_t nbytes, void *stream);

/* The same with the width as an argument (8, 16, 32 or 64). */
ppc_status ppc_pospopcnt(unsigned width, uint64_t *counts, const void *buf, size_t nbytes,
                         void *stream);

/* ------------------------------------------------------------------------
 * Launch geometry of the plain call.  `waves` caps the number of wavefronts
 * the grid holds (0 = the library default: 8 per compute unit);
 * `waves_per_block` is 2, 4 or 8 (default 8).  Applies to later plain calls
 * from any thread on any device.  Returns PPC_EINVAL for values out of range.
 * ---------------------------------------------------------------------- */
ppc_status ppc_set_plain_geometry(unsigned waves, unsigned waves_per_block);
ppc_status ppc_get_plain_geometry(unsigned *waves, unsigned *waves_per_block);

/* ------------------------------------------------------------------------
 * Read roofline: the "dummy" kernel of the paper's benchmark (Section 5,
 * Table "Benchmarked algorithms"), which sums the input and adds the sum to
 * an output.  *sink (device, one uint64) += sum of the little-endian 64-bit
 * words of buf[0..nbytes) mod 2^64; `buf` must be 16-byte aligned and
 * nbytes a multiple of 16 KiB (whole tiles).  Same load pattern and launch
 * geometry as the plain pospopcnt call: it measures the bandwidth that call
 * can reach.
 * ---------------------------------------------------------------------- */
ppc_status ppc_read_roofline(uint64_t *sink, const void *buf, size_t nbytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PPC_H */
