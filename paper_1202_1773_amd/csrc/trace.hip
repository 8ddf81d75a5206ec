// trace.hip -- host-side tracing of the library: the FFST_LOG text log and
// roctx ranges around the C ABI calls and kernel launches.
#include "internal.hpp"

#include <rocprofiler-sdk-roctx/roctx.h>
#include <unistd.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

namespace {

struct LogSink {
  int level = 0;
  FILE* fp = nullptr;
  std::mutex mu;
};

// FFST_LOG = "", "0"         : off
//            "1", "2"         : that level, on stderr
//            "<level>:<path>" : that level, appended to <path>
//            anything else    : a path, level 1
LogSink& sink() {
  static LogSink* s = [] {
    LogSink* k = new LogSink;
    const char* v = std::getenv("FFST_LOG");
    if (!v || !*v || std::strcmp(v, "0") == 0) return k;
    const char* path = nullptr;
    if (v[0] >= '1' && v[0] <= '9' && (v[1] == '\0' || v[1] == ':')) {
      k->level = v[0] - '0';
      if (v[1] == ':' && v[2]) path = v + 2;
    } else {
      k->level = 1;
      path = v;
    }
    k->fp = stderr;
    if (path) {
      FILE* f = std::fopen(path, "a");
      if (f)
        k->fp = f;
      else
        std::fprintf(stderr, "ffst: cannot open FFST_LOG file %s; logging to stderr\n", path);
    }
    return k;
  }();
  return *s;
}

}  // namespace

int ffst::log_level() { return sink().level; }

void ffst::log_line(int level, const char* fmt, ...) {
  LogSink& k = sink();
  if (level > k.level || !k.fp) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::lock_guard<std::mutex> lk(k.mu);
  std::fprintf(k.fp, "ffst[%d] %s\n", (int)getpid(), buf);
  std::fflush(k.fp);
}

ffst::Range::Range(const char* name) { (void)roctxRangePushA(name); }
ffst::Range::~Range() { (void)roctxRangePop(); }
