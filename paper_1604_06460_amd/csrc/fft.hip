// QFT emulation (Sec. III-B): replaced in the next change by the in-place
// multi-pass FFT.
#include "qs_internal.h"

extern "C" int qs_emulate_qft(qs_handle h, int q_lo, int m, int inverse)
{
    (void)inverse;
    qs::clear_error();
    if (!h) return qs::fail(QS_EINVAL, "NULL handle");
    if (m < 1 || q_lo < 0 || q_lo + m > h->n) return qs::fail(QS_EINVAL, "QFT field outside the state");
    return qs::fail(QS_EUNSUPPORTED, "QFT emulation not built yet");
}
