// Batched solves and the request server (see server.hip).
#pragma once

#include "core.hpp"

namespace rid {

rid_status batch_run(rid_context* ctx, int n, rid_problem* const* probs, const rid_request* reqs,
                     rid_result* results);

// Device bytes a request needs beyond its problem's tensors (estimate used
// for admission).
uint64_t request_footprint(const rid_problem* P, const rid_request& r);

rid_server* server_create(rid_context* ctx, const rid_server_opts& o);
rid_status server_submit(rid_server* s, rid_problem* P, const rid_request* r, rid_result* res, uint64_t* ticket);
rid_status server_poll(rid_server* s, uint64_t ticket);
rid_status server_wait(rid_server* s, uint64_t ticket, int timeout_ms);
rid_status server_cancel(rid_server* s, uint64_t ticket);
void server_destroy(rid_server* s);

}  // namespace rid
