// Streaming interface (filled in with the chunk pipeline).
#include "ecc_internal.h"

using namespace ecc;

extern "C" {

int ecc_stream_begin(const ecc_dims *full_dims, ecc_dtype dtype, void *stream, ecc_stream **out) {
    (void)full_dims; (void)dtype; (void)stream; (void)out;
    set_error("streaming is not available in this build");
    return ECC_E_UNSUPPORTED;
}

int ecc_stream_push_chunk(ecc_stream *st, const void *planes, int64_t n_planes) {
    (void)st; (void)planes; (void)n_planes;
    set_error("streaming is not available in this build");
    return ECC_E_UNSUPPORTED;
}

int ecc_stream_finish(ecc_stream *st, ecc_curve *curve) {
    (void)st; (void)curve;
    set_error("streaming is not available in this build");
    return ECC_E_UNSUPPORTED;
}

void ecc_stream_abort(ecc_stream *st) { (void)st; }

}
