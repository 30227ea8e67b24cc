// Error reporting shared by the library's translation units.
#pragma once

namespace mmlttb {

// Records a printf-style message as the calling thread's last error (read by
// mmlttb_last_error) and returns `code`.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

} // namespace mmlttb
