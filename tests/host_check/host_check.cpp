// Host-side checks of the C ABI under AddressSanitizer and UBSan: every call
// here returns before any launch (sizes, layouts, status strings, argument
// and workspace checks), so no GPU is needed.  Exit status 0 when every
// check holds; a sanitizer report aborts with its own status.
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "cgd_enkf.h"

static int failures = 0;
#define CHECK(cond)                                                       \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

int main() {
  const int ns[] = {1, 7, 40, 4096, 65536};
  const int ms[] = {1, 5, 33, 2048, 16384};
  const int Ns[] = {2, 5, 16, 33, 64, 100, 128, 160};
  const int ks[] = {1, 4};
  long shapes = 0;
  for (int n : ns)
    for (int m : ms)
      for (int N : Ns)
        for (int k : ks)
          for (int prec = 0; prec < 4; ++prec) {
            for (int mode = 0; mode < 4; ++mode) {
              const size_t b = cgd_enkf_workspace_bytes(n, m, N, k, prec, mode);
              CHECK(b % 256 == 0);
            }
            CHECK(cgd_layout_selfcheck(n, m, N, k, prec) == 0);
            const size_t g = cgd_enkf_gain_workspace_bytes(n, m, N, k, prec);
            CHECK((g == 0) == (prec > 1 || N > 128));
            ++shapes;
          }
  CHECK(cgd_layout_selfcheck(10, 10, 1, 1, 0) == -1);
  CHECK(cgd_enkf_workspace_bytes(0, 10, 10, 1, 0, 0) == 0);
  for (int s = -8; s <= 1; ++s) CHECK(std::strlen(cgd_status_string(s)) > 0);

  // argument and workspace checks, with pointers that are never dereferenced
  cgd_options opt;
  cgd_options_default(&opt);
  void* d = reinterpret_cast<void*>(uintptr_t{256});
  const int32_t* di = reinterpret_cast<const int32_t*>(d);
  CHECK(cgd_enkf_analysis(40, 20, 1, 1, d, d, di, d, d, d, nullptr, 1e-6, 10, &opt, d, 1u << 30,
                          nullptr, nullptr) == CGD_ERR_ARG);
  CHECK(cgd_enkf_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, -1.0, 10, &opt, d, 1u << 30,
                          nullptr, nullptr) == CGD_ERR_ARG);
  CHECK(cgd_enkf_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, 1e-6, 10, &opt, d, 16,
                          nullptr, nullptr) == CGD_ERR_WORKSPACE);
  CHECK(cgd_enkf_reduced_analysis(40, 0, 20, 1, d, d, di, d, d, d, nullptr, 1e-6, 10, &opt, d,
                                  1u << 30, nullptr, nullptr) == CGD_ERR_ARG);
  CHECK(cgd_senkf_analysis(40, 20, 1, 1, d, d, di, d, d, d, nullptr, &opt, d, 1u << 30, nullptr,
                           nullptr) == CGD_ERR_ARG);
  CHECK(cgd_senkf_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, &opt, d, 16, nullptr,
                           nullptr) == CGD_ERR_WORKSPACE);
  CHECK(cgd_enkf_gain_analysis(40, 20, 130, 1, d, d, di, d, d, d, nullptr, 1e-6, 10, &opt,
                               nullptr, nullptr, d, 1u << 30, nullptr,
                               nullptr) == CGD_ERR_UNSUPPORTED);
  CHECK(cgd_enkf_gain_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, 1e-6, -1, &opt, nullptr,
                               nullptr, d, 1u << 30, nullptr, nullptr) == CGD_ERR_ARG);
  cgd_options bad = opt;
  bad.prec = 9;
  CHECK(cgd_enkf_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, 1e-6, 10, &bad, d, 1u << 30,
                          nullptr, nullptr) == CGD_ERR_ARG);
  bad.prec = CGD_MIXED_BF16;
  CHECK(cgd_senkf_analysis(40, 20, 20, 1, d, d, di, d, d, d, nullptr, &bad, d, 1u << 30, nullptr,
                           nullptr) == CGD_ERR_UNSUPPORTED);
  std::printf("host checks: %ld shapes, %d failures\n", shapes, failures);
  return failures ? 1 : 0;
}
