// Serving front end: placeholder until the continuous-batching scheduler lands.
#include "../../include/wfa.h"
#include "internal.h"

extern "C" int wfa_server_open(wfa_ctx*, const wfa_server_cfg*, wfa_server** out) {
    if (out) *out = nullptr;
    return WFA_E_INVAL;
}
extern "C" int wfa_server_submit(wfa_server*, const wfa_request*, uint64_t*) { return WFA_E_INVAL; }
extern "C" int wfa_server_poll(wfa_server*, uint64_t, int64_t, wfa_result*) { return WFA_E_INVAL; }
extern "C" int wfa_server_release(wfa_server*, uint64_t) { return WFA_E_INVAL; }
extern "C" size_t wfa_server_estimate_bytes(const wfa_server*, const wfa_request*) { return 0; }
extern "C" int wfa_server_close(wfa_server*) { return WFA_E_INVAL; }
