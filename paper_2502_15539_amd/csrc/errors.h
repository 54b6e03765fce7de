// Error reporting shared by the C ABI layer and the host builder: records a
// message for ptrhash_last_error() on the calling thread, returns code.
#pragma once

namespace ptrhash {
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
}
