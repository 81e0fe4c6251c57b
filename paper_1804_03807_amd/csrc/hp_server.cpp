// Serving loop of libhomotopy (continuous batching over the persistent
// tracker).  Placeholder entry points until the loop lands.
#include <string>

#include "homotopy.h"

struct hp_server {
  int unused;
};

extern "C" {
int hp_server_create(hp_context *, size_t, hp_server **out) {
  if (out) *out = nullptr;
  return HP_E_INVALID_ARG;
}
int hp_server_submit(hp_server *, const hp_system *, hp_c64, const hp_tolerances *, int64_t *) {
  return HP_E_INVALID_ARG;
}
int hp_server_poll(hp_server *, int64_t, int32_t *) { return HP_E_INVALID_ARG; }
int hp_server_wait(hp_server *, int64_t, hp_c64 *, int32_t *, hp_path_stats *, double *) {
  return HP_E_INVALID_ARG;
}
int hp_server_peak_bytes(hp_server *, size_t *) { return HP_E_INVALID_ARG; }
void hp_server_destroy(hp_server *) {}
}
