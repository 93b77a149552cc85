// Host-only checks of libpss's argument validation, planning and workspace
// arithmetic, built with the address and undefined-behaviour sanitizers
// (host code only; no kernel is launched and no GPU is needed).  Exits 0 when
// every check holds; a sanitizer report or a failed check exits non-zero.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pss.h"

namespace pss {
bool inject_fault(int kind);
}

static int failures = 0;
#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

int main() {
  // every status has a name; the thread's last error starts empty
  for (int s = 0; s <= 8; ++s) CHECK(std::strlen(pss_status_string((pss_status)s)) > 0);
  CHECK(pss_last_error(nullptr) != nullptr);

  // argument validation (addresses are compared, never dereferenced)
  char *a = (char *)0x100000, *b = (char *)0x200000;
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, a, b, nullptr, nullptr, 100, 0, 0, SIZE_MAX) == PSS_OK);
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, a, a + 8, nullptr, nullptr, 100, 0, 0, SIZE_MAX) ==
        PSS_ERR_INVALID);  // overlap
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, nullptr, b, nullptr, nullptr, 1, 0, 0, SIZE_MAX) ==
        PSS_ERR_INVALID);
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, nullptr, nullptr, nullptr, nullptr, 0, 0, 0, SIZE_MAX) ==
        PSS_OK);  // n = 0 needs no pointers
  CHECK(pss_validate((pss_key_t)9, PSS_VAL_NONE, a, b, nullptr, nullptr, 1, 0, 0, SIZE_MAX) ==
        PSS_ERR_INVALID);
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, a, b, nullptr, nullptr, 1, 4, 0, SIZE_MAX) ==
        PSS_ERR_INVALID);  // one of n_B, n_P zero
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, a, b, nullptr, nullptr, (uint64_t)1 << 31, 0, 0,
                     SIZE_MAX) == PSS_ERR_UNSUPPORTED);
  CHECK(pss_validate(PSS_U64, PSS_VAL_U32, a, b, nullptr, (uint32_t *)0x300000, 10, 0, 0,
                     SIZE_MAX) == PSS_ERR_INVALID);  // null vals_in
  CHECK(pss_validate(PSS_I64, PSS_VAL_NONE, a, b, nullptr, nullptr, 100, 0, 0, 16) ==
        PSS_ERR_WORKSPACE);

  // workspace sizes and plans over many sizes, both modes and all key types
  std::vector<uint64_t> ns = {0, 1, 2, 3, 100, 8191, 8192, 8193, 65536, 1000003, (uint64_t)1 << 24,
                              ((uint64_t)1 << 28) + 7, (uint64_t)1 << 30, PSS_MAX_KEYS};
  char buf[4096];
  for (int kt = 0; kt <= 5; ++kt) {
    for (int v = 0; v <= 1; ++v) {
      size_t prev = 0;
      for (uint64_t n : ns) {
        size_t ws = 0;
        CHECK(pss_workspace_bytes(nullptr, (pss_key_t)kt, (pss_val_t)v, n, 0, 0, &ws) == PSS_OK);
        CHECK(ws >= prev);
        prev = ws;
        CHECK(pss_plan_describe((pss_key_t)kt, (pss_val_t)v, n, 0, 0, buf, sizeof buf) == PSS_OK);
        CHECK(std::strstr(buf, "\"mode\": \"auto\"") != nullptr);
        for (uint32_t nb : {1u, 3u, 64u, 256u, 2048u}) {
          size_t wp = 0;
          const pss_status st =
              pss_workspace_bytes(nullptr, (pss_key_t)kt, (pss_val_t)v, n, nb, 64, &wp);
          CHECK(st == PSS_OK || st == PSS_ERR_UNSUPPORTED);
          if (st == PSS_OK)
            CHECK(pss_plan_describe((pss_key_t)kt, (pss_val_t)v, n, nb, 64, buf, sizeof buf) ==
                  PSS_OK);
          size_t wr = 0;
          const pss_status sr =
              pss_psrs_workspace_bytes(nullptr, (pss_key_t)kt, (pss_val_t)v, n, nb, 64, &wr);
          CHECK(sr == PSS_OK || sr == PSS_ERR_UNSUPPORTED);
        }
        size_t wrec = 0;
        CHECK(pss_records_workspace_bytes(nullptr, (pss_key_t)kt, n, &wrec) == PSS_OK);
        for (uint32_t segs : {1u, 7u, 4096u}) {
          for (uint32_t f : {0u, 5u, 6u}) {
            pss_tuning tu{2048, 4096, 0, f, 0};
            size_t wseg = 0;
            CHECK(pss_segmented_workspace_bytes(nullptr, (pss_key_t)kt, (pss_val_t)v, n, segs, &tu,
                                                &wseg) == PSS_OK);
          }
          pss_tuning bad{2048, 4096, 0, 4, 0};
          size_t wb = 0;
          CHECK(pss_segmented_workspace_bytes(nullptr, (pss_key_t)kt, (pss_val_t)v, n, segs, &bad,
                                              &wb) == PSS_ERR_INVALID);
        }
      }
    }
  }
  // a buffer too small for the plan is refused, not overrun
  char tiny[8];
  CHECK(pss_plan_describe(PSS_I64, PSS_VAL_NONE, (uint64_t)1 << 28, 0, 0, tiny, sizeof tiny) ==
        PSS_ERR_INVALID);

  // fault injection: after = k lets k operations through, fails the next one
  CHECK(pss_debug_inject(PSS_INJECT_LAUNCH, 2) == PSS_OK);
  CHECK(!pss::inject_fault(1));
  CHECK(!pss::inject_fault(1));
  CHECK(pss::inject_fault(1));
  CHECK(!pss::inject_fault(1));  // used up
  CHECK(pss_debug_inject(PSS_INJECT_ALLOC, 0) == PSS_OK);
  CHECK(!pss::inject_fault(1));  // the other kind is not affected
  CHECK(pss_debug_inject(PSS_INJECT_NONE, 0) == PSS_OK);
  CHECK(!pss::inject_fault(2));  // disarmed
  CHECK(pss_debug_inject((pss_inject_t)7, 0) == PSS_ERR_INVALID);

  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("host ABI checks passed\n");
  return 0;
}
