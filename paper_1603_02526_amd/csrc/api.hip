// Library-wide C ABI pieces: per-thread error messages, version, and the
// device probe used before any allocation.
#include "internal.h"

namespace {
thread_local std::string g_err;
}

namespace admmi {

admm_status set_err(admm_status s, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void clear_err() { g_err.clear(); }

admm_status probe_device(int device) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return set_err(ADMM_E_NO_DEVICE, "no HIP device available");
  }
  if (device < 0 || device >= n)
    return set_err(ADMM_E_ARG, "device %d out of range [0,%d)", device, n);
  return ADMM_OK;
}

}  // namespace admmi

extern "C" {

const char* admm_last_error(void) { return g_err.c_str(); }

int32_t admm_abi_version(void) { return 1; }

}  // extern "C"
