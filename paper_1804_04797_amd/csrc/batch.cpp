// Batched persistent execution (sv_batch_*).
#include "qsv_internal.h"

using namespace qsv;

extern "C" {

qsv_status sv_batch_create(const qsv_circuit *const *circs, const uint64_t *branch_ids,
                           size_t count, const qsv_fuse_opts *opts, qsv_batch **out) {
    (void)circs; (void)branch_ids; (void)count; (void)opts;
    if (out) *out = nullptr;
    return fail(QSV_EUNSUPPORTED, "sv_batch_create: not built yet");
}

qsv_status sv_batch_run(qsv_batch *b, void *const *amps_dev, int init_plus,
                        const uint64_t *bitstrings_dev, size_t m, void *amp_table_dev,
                        void *stream) {
    (void)b; (void)amps_dev; (void)init_plus; (void)bitstrings_dev; (void)m; (void)amp_table_dev;
    (void)stream;
    return fail(QSV_EUNSUPPORTED, "sv_batch_run: not built yet");
}

void sv_batch_destroy(qsv_batch *b) { (void)b; }

}
