// CPU unit test of pso_guard.hpp: whatever an entry point's body throws
// becomes a status code instead of crossing the C ABI.  The allocation
// failure is real: the address space is capped with RLIMIT_AS and a body
// then asks for more than that.  Prints "ok" and exits 0 on success.
#include <sys/resource.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../paper_2205_01313_amd/csrc/pso_guard.hpp"

static char g_msg[512];

int pso_internal_fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL line %d: %s (%s)\n", __LINE__, #c, g_msg);     \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main()
{
    // a body that returns normally passes its status through
    CHECK(pso::guarded([] { return PSO_OK; }) == PSO_OK);
    CHECK(pso::guarded([] { return PSO_ESTATE; }) == PSO_ESTATE);
    // thrown exceptions become statuses
    CHECK(pso::guarded([]() -> int { throw std::bad_alloc(); }) == PSO_ENOMEM);
    CHECK(pso::guarded([]() -> int { throw std::runtime_error("boom"); }) == PSO_EDEVICE);
    CHECK(std::strstr(g_msg, "boom") != nullptr);
    CHECK(pso::guarded([]() -> int { throw 42; }) == PSO_EDEVICE);
    // a container asked for more elements than it can hold
    CHECK(pso::guarded([]() -> int {
              std::vector<int> v;
              v.reserve(v.max_size() + 1);
              return PSO_OK;
          }) == PSO_ENOMEM);
    // a real allocation failure: cap the address space, then allocate beyond it
    rlimit lim{};
    CHECK(getrlimit(RLIMIT_AS, &lim) == 0);
    lim.rlim_cur = rlim_t(512) << 20;
    CHECK(setrlimit(RLIMIT_AS, &lim) == 0);
    int rc = pso::guarded([]() -> int {
        std::vector<char> big(size_t(2) << 30, 1);
        return big[12345] == 1 ? PSO_OK : PSO_EINVAL;
    });
    CHECK(rc == PSO_ENOMEM);
    CHECK(std::strstr(g_msg, "allocation") != nullptr);
    // and the process carries on: a small allocation still works
    std::string s(1000, 'x');
    CHECK(s.size() == 1000);
    std::printf("ok\n");
    return 0;
}
