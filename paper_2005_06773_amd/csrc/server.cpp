#include "runtime.h"
extern "C" mhc_status mhc_server_start(mhc_ctx *, const mhc_server_cfg *, mhc_server **) { return MHC_E_DEVICE; }
extern "C" mhc_status mhc_submit(mhc_server *, int32_t, const mhc_scene *, mhc_result *, uint64_t *) { return MHC_E_DEVICE; }
extern "C" mhc_status mhc_wait(mhc_server *, uint64_t, int64_t, mhc_timing *) { return MHC_E_DEVICE; }
extern "C" mhc_status mhc_server_stats(mhc_server *, mhc_stats *) { return MHC_E_DEVICE; }
extern "C" mhc_status mhc_server_stop(mhc_server *) { return MHC_E_DEVICE; }
