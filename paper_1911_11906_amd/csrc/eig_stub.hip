// Placeholder entry points for the eigensolver stages (replaced by eig.hip).
#include "internal.h"
extern "C" {
int fl_eigensolve(fl_op* op, int, const fl_eig_opts*, fl_eig_info*) { return fl_fail(op ? op->ctx : nullptr, FL_EINVAL, "not built"); }
int fl_dstedc(fl_ctx* c, int64_t, double*, double*, double*, int64_t) { return fl_fail(c, FL_EINVAL, "not built"); }
int fl_dsytrd_2stage(fl_ctx* c, int64_t, double*, int64_t, int, double*, double*, double*, int64_t) { return fl_fail(c, FL_EINVAL, "not built"); }
int fl_dsyevd(fl_ctx* c, int64_t, double*, int64_t, int, double*, double*, int64_t) { return fl_fail(c, FL_EINVAL, "not built"); }
}
