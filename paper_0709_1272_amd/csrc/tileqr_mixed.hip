// Tiled QR kernels with split-precision LARFB / SSRFB products, instantiated
// for one arithmetic per object: the build compiles this file once for each
// value of TQ_PREC (1 BF16 x2, 2 FP16 x2, 3 BF16 x3), always with ib = 32.
// Reflectors and T are formed in FP64; the block-reflector products (in
// LARFB, SSRFB and the trailing updates inside GEQRT / TSQRT) are split.
#define TQ_OPAQUE_TID 1
#include "tileqr_tile.h"

#ifndef TQ_PREC
#error "TQ_PREC must name the split arithmetic (1, 2 or 3)"
#endif

namespace tq {

static_assert(TQ_PREC == PREC_BF16X2 || TQ_PREC == PREC_FP16X2 || TQ_PREC == PREC_BF16X3, "TQ_PREC");

#define TQ_MX_DISPATCH(nb, CALL)                   \
    do {                                           \
        if (nb == 64) { CALL(64); }                \
        else if (nb == 128) { CALL(128); }         \
        else if (nb == 256) { CALL(256); }         \
    } while (0)

template <int PREC>
hipError_t launch_serial_mx(int nb, const MatDev &M, const int *status, hipStream_t st)
{
#define TQ_CALL(NB) return serial_impl<NB, 32, PREC>(M, status, st)
    TQ_MX_DISPATCH(nb, TQ_CALL);
#undef TQ_CALL
    return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_worker_mx(int nb, const SchedDev &S, int workers, hipStream_t st)
{
#define TQ_CALL(NB) return worker_impl<NB, 32, PREC>(S, workers, st)
    TQ_MX_DISPATCH(nb, TQ_CALL);
#undef TQ_CALL
    return hipErrorInvalidValue;
}

template <int PREC>
int worker_occupancy_mx(int nb)
{
#define TQ_CALL(NB) return worker_occupancy_impl<NB, 32, PREC>()
    TQ_MX_DISPATCH(nb, TQ_CALL);
#undef TQ_CALL
    return 1;
}

template hipError_t launch_serial_mx<TQ_PREC>(int, const MatDev &, const int *, hipStream_t);
template hipError_t launch_worker_mx<TQ_PREC>(int, const SchedDev &, int, hipStream_t);
template int worker_occupancy_mx<TQ_PREC>(int);

}  // namespace tq
