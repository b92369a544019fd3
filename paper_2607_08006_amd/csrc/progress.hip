// Persistent progress kernel and trace-driven serving (in progress).
#include "runtime.hpp"

extern "C" {
int shmemx_progress_start(const shmemx_progress_cfg_t *, void *) { return SHMEMX_ERR_UNSUPPORTED; }
int shmemx_progress_submit(const shmemx_desc_t *, uint64_t *) { return SHMEMX_ERR_UNSUPPORTED; }
int shmemx_progress_poll(uint64_t, shmemx_completion_t *) { return SHMEMX_ERR_UNSUPPORTED; }
int shmemx_progress_stop(int) { return SHMEMX_ERR_UNSUPPORTED; }
int shmemx_serve_run(const shmemx_request_t *, size_t, int, uint64_t, uint64_t, uint64_t, uint64_t *, uint64_t *,
                     shmemx_completion_t *, shmemx_serve_stats_t *)
{
    return SHMEMX_ERR_UNSUPPORTED;
}
}
