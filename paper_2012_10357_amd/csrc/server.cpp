// Serving entry points (continuous batching) -- filled in below.
#include "host_common.h"

extern "C" {
pr_status pr_server_create(const pr_server_opts*, pr_server**) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_add_scene(pr_server*, pr_scene*, uint32_t*) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_submit(pr_server*, const pr_request*, uint64_t*) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_wait(pr_server*, uint64_t, uint32_t, pr_request_result*) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_release(pr_server*, uint64_t) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_stats_get(pr_server*, pr_server_stats*) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
pr_status pr_server_destroy(pr_server*) { return pr::set_error(PR_ERR_UNSUPPORTED, "server not built yet"); }
}
