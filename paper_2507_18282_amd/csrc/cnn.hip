// Learned warm start for the implicit solves (see cnn.hip's later revision).
#include "op.h"

namespace ew {

ew_status cnn_predict(Op* op, const double* wcur, const double* wprev, double* guess_S) {
    (void)op; (void)wcur; (void)wprev; (void)guess_S;
    return fail(EW_ERR_UNSUPPORTED, "learned predictor not available");
}

}  // namespace ew
