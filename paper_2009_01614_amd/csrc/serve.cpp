// Serving loop (work in progress).
#include "internal.h"
extern "C" {
isax_server* isax_server_create(isax_index* const*, int32_t, const isax_server_options*) {
    isax::set_error(ISAX_EINVAL, "server not available in this build");
    return nullptr;
}
int isax_server_submit(isax_server*, int32_t, const float*, int32_t, uint64_t) { return ISAX_EINVAL; }
int isax_server_poll(isax_server*, isax_result*, int32_t, int32_t) { return ISAX_EINVAL; }
int64_t isax_server_pending(isax_server*) { return 0; }
void isax_server_destroy(isax_server*) {}
}
