// temporary
#include "qt_host.hpp"
extern "C" {
qt_status qt_job_create(qt_context*, const qt_physics*, const qt_ttable*, const qt_init*, const qt_batch*, int64_t, qt_job**) { return QT_EINVAL; }
qt_status qt_job_advance(qt_job*, int64_t, void*) { return QT_EINVAL; }
qt_status qt_job_done(qt_job*, int32_t*) { return QT_EINVAL; }
qt_status qt_job_state_bytes(qt_job*, size_t*) { return QT_EINVAL; }
qt_status qt_job_save(qt_job*, void*, void*) { return QT_EINVAL; }
qt_status qt_job_load(qt_job*, const void*, void*) { return QT_EINVAL; }
qt_status qt_job_results(qt_job*, const qt_results*, void*) { return QT_EINVAL; }
qt_status qt_job_destroy(qt_job*) { return QT_EINVAL; }
qt_status qt_server_create(qt_context*, const qt_server_cfg*, qt_server**) { return QT_EINVAL; }
qt_status qt_submit(qt_server*, const qt_physics*, const qt_ttable*, const qt_init*, const qt_batch*, uint64_t*) { return QT_EINVAL; }
qt_status qt_poll(qt_server*, uint64_t, int32_t*) { return QT_EINVAL; }
qt_status qt_wait(qt_server*, uint64_t, const qt_results*, double) { return QT_EINVAL; }
qt_status qt_cancel(qt_server*, uint64_t) { return QT_EINVAL; }
qt_status qt_server_stats(qt_server*, qt_stats*) { return QT_EINVAL; }
qt_status qt_server_destroy(qt_server*) { return QT_EINVAL; }
}
