// Placeholder entry points of the adjoint and batched forms.
#include "../../include/qsv.h"

extern "C" {
qsv_status qsv_adjoint_gradient(qsv_sim *, const qsv_circuit *, const qsv_pauli_sum *, double *,
                                double *) {
    return QSV_EUNSUPPORTED;
}
qsv_status qsv_batch_create(int32_t, const qsv_circuit *, const qsv_pauli_sum *,
                            const qsv_batch_options *, qsv_batch **) {
    return QSV_EUNSUPPORTED;
}
qsv_status qsv_batch_run(qsv_batch *, double *) { return QSV_EUNSUPPORTED; }
qsv_status qsv_batch_info(const qsv_batch *, int32_t *, int32_t *, double *) {
    return QSV_EUNSUPPORTED;
}
qsv_status qsv_batch_destroy(qsv_batch *) { return QSV_EUNSUPPORTED; }
}
