// Batched search and the search server.
#include "ffa_internal.h"

using namespace ffa;

extern "C" ffa_status ffa_batch_workspace(int32_t n, const ffa_plan* plans, size_t* ws_bytes) {
  (void)n; (void)plans; (void)ws_bytes;
  return fail(FFA_ERR_UNSUPPORTED, "batched search not built yet");
}

extern "C" ffa_status ffa_search_batch(int32_t n, const ffa_plan* plans, const void* const* d_series,
                                       float* const* d_snr, int32_t* const* d_width, void* d_ws,
                                       size_t ws_bytes, void* stream) {
  (void)n; (void)plans; (void)d_series; (void)d_snr; (void)d_width; (void)d_ws; (void)ws_bytes; (void)stream;
  return fail(FFA_ERR_UNSUPPORTED, "batched search not built yet");
}

extern "C" ffa_status ffa_server_create(size_t budget, int32_t n_streams, ffa_server* out) {
  (void)budget; (void)n_streams; (void)out;
  return fail(FFA_ERR_UNSUPPORTED, "server not built yet");
}
extern "C" ffa_status ffa_server_submit(ffa_server s, ffa_plan p, const void* series, int is_device,
                                        int64_t* ticket) {
  (void)s; (void)p; (void)series; (void)is_device; (void)ticket;
  return fail(FFA_ERR_UNSUPPORTED, "server not built yet");
}
extern "C" ffa_status ffa_server_wait(ffa_server s, int64_t ticket, int64_t timeout_us, float* snr,
                                      int32_t* width, double* latency) {
  (void)s; (void)ticket; (void)timeout_us; (void)snr; (void)width; (void)latency;
  return fail(FFA_ERR_UNSUPPORTED, "server not built yet");
}
extern "C" ffa_status ffa_server_destroy(ffa_server s) {
  (void)s;
  return fail(FFA_ERR_UNSUPPORTED, "server not built yet");
}
