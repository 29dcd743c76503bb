// wf_server.cpp -- serving front end (admission by HBM budget, continuous batching).
#include "../../include/wf.h"

struct wf_server {};

extern "C" wf_status wf_server_create(wf_ctx*, const wf_server_opts*, wf_server**) { return WF_EUNSUPPORTED; }
extern "C" wf_status wf_submit(wf_server*, const wf_request*, uint64_t*) { return WF_EUNSUPPORTED; }
extern "C" wf_status wf_poll(wf_server*, uint64_t, wf_result*) { return WF_EUNSUPPORTED; }
extern "C" wf_status wf_release(wf_server*, uint64_t) { return WF_EUNSUPPORTED; }
extern "C" wf_status wf_server_destroy(wf_server*) { return WF_EUNSUPPORTED; }
extern "C" wf_status wf_server_memory(wf_server*, int64_t*, int64_t*) { return WF_EUNSUPPORTED; }
