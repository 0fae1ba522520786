// A fixed device area for the entry points that allocate nothing.
//
// The array below lives in the library's code object: each GPU the library
// runs on holds its own copy, at its own address, from the first use of the
// library on that device until the process ends.  Host code never passes
// the array's name to a kernel (on the host the name is only a stand-in
// for the symbol); it asks the runtime for the device address once per
// device, with that device current, and uses that address everywhere.
//
// Every call on one GPU shares that GPU's area, so calls that overlap on
// one GPU (two host threads, or two streams with work in flight) race; the
// area keeps whatever the last call left in it, and each call clears what
// it needs cleared.
#include <map>
#include <mutex>

#include "dg_host.h"

namespace dg {

static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static std::map<int, void*> g_noalloc_ptr;   // device -> address of its copy of the area

hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr.count(device)) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_noalloc_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_area(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(device);
  return it == g_noalloc_ptr.end() ? nullptr : it->second;
}

}  // namespace dg
