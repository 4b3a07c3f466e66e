/* couple_hbmref.h -- streaming reference kernels of libcouple.so.
 *
 * Not part of the coupling method: three plain passes over a device buffer
 * (read, write, copy) in the access forms that run fastest on this chip (one
 * 16-byte element per thread, non-temporal loads, one workgroup per 256
 * elements).  The rates they sustain are the practical HBM ceiling against
 * which the coupling kernels' bandwidths are read, beside the vendor peak.
 *
 * Element counts are in 16-byte units; pointers are device pointers, 16-byte
 * aligned (the read's flag: 4-byte aligned), owned by the caller; stream is a hipStream_t (NULL: the default
 * stream).  Calls are asynchronous on the stream.
 */
#ifndef COUPLE_HBMREF_H
#define COUPLE_HBMREF_H

#include <stdint.h>

#include "couple.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    COUPLE_HBMREF_READ = 0,   /* reads src[0 .. n16) and sets the int32 *dst to 1 if any of its
                                 4 n16 floats is NaN or infinite (left as it is otherwise: the
                                 caller clears it); a scan for non-finite values */
    COUPLE_HBMREF_WRITE = 1,  /* writes the float `value` to all 4 n16 floats of dst; src unused */
    COUPLE_HBMREF_COPY = 2    /* copies src[0 .. n16) to dst */
};

/* One pass of `kind` over n16 16-byte elements.  Returns COUPLE_OK, or
 * COUPLE_EINVAL for an unknown kind, n16 < 0, a NULL or misaligned pointer the
 * kind uses (n16 = 0 is a no-op), COUPLE_EHIP when the launch fails. */
int couple_hbmref(int kind, const void *src, void *dst, int64_t n16, float value, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* COUPLE_HBMREF_H */
