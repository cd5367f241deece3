// HBM-footprint admission ledger of include/nsr.h (ns_ledger_*), and the
// footprint of one solve.  Host code only: a budget, the bytes in service
// and their peak, under a mutex, so serving loops on any number of host
// threads can admit and release requests through one ledger.
#include <mutex>
#include <new>

#include "nsr.h"
#include "nsr_internal.h"

struct ns_ledger {
  std::mutex mu;
  size_t budget = 0;
  size_t in_use = 0;
  size_t peak = 0;
  uint64_t admitted = 0;
  uint64_t refused = 0;
};

extern "C" {

int ns_ledger_create(size_t budget_bytes, ns_ledger** out) {
  if (!out) {
    nsr::ns_set_error("null out");
    return NS_EINVAL;
  }
  *out = nullptr;
  if (budget_bytes == 0) {
    nsr::ns_set_error("budget must be > 0");
    return NS_EINVAL;
  }
  ns_ledger* L = new (std::nothrow) ns_ledger();
  if (!L) {
    nsr::ns_set_error("host allocation failed");
    return NS_ENOMEM;
  }
  L->budget = budget_bytes;
  *out = L;
  return NS_OK;
}

int ns_ledger_admit(ns_ledger* L, size_t bytes) {
  if (!L) {
    nsr::ns_set_error("null ledger");
    return NS_EINVAL;
  }
  std::lock_guard<std::mutex> g(L->mu);
  if (bytes > L->budget) {
    nsr::ns_set_error("footprint larger than the whole budget");
    return NS_EINVAL;
  }
  if (bytes > L->budget - L->in_use) {
    ++L->refused;
    nsr::ns_set_error("over the HBM budget");
    return NS_ENOMEM;
  }
  L->in_use += bytes;
  if (L->in_use > L->peak) L->peak = L->in_use;
  ++L->admitted;
  return NS_OK;
}

int ns_ledger_release(ns_ledger* L, size_t bytes) {
  if (!L) {
    nsr::ns_set_error("null ledger");
    return NS_EINVAL;
  }
  std::lock_guard<std::mutex> g(L->mu);
  if (bytes > L->in_use) {
    nsr::ns_set_error("release of more bytes than are in service");
    return NS_EINVAL;
  }
  L->in_use -= bytes;
  return NS_OK;
}

int ns_ledger_query(ns_ledger* L, size_t* in_use, size_t* peak, size_t* budget,
                    uint64_t* admitted, uint64_t* refused) {
  if (!L) {
    nsr::ns_set_error("null ledger");
    return NS_EINVAL;
  }
  std::lock_guard<std::mutex> g(L->mu);
  if (in_use) *in_use = L->in_use;
  if (peak) *peak = L->peak;
  if (budget) *budget = L->budget;
  if (admitted) *admitted = L->admitted;
  if (refused) *refused = L->refused;
  return NS_OK;
}

int ns_ledger_destroy(ns_ledger* L) {
  delete L;
  return NS_OK;
}

size_t ns_solve_footprint(int64_t n, int precision, int composite) {
  if (n < 1) return 0;
  const size_t ws = ns_workspace_bytes(n, precision, composite);
  if (ws == 0) return 0;
  return ws + ((size_t)n * (size_t)n + 2 * (size_t)n) * sizeof(double);
}

}  // extern "C"
