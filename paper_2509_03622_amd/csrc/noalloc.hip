// Fixed device scratch for the entry point that allocates nothing
// (nosdd_precond_apply_noalloc).
//
// The array below lives in the code object: every GPU the library runs on
// holds its own copy from module load until the process ends.  In host code
// the array's name is only a host-side stand-in, so its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// when a context is created there, and only that address is ever handed to
// kernels.  Every call on one GPU shares that GPU's copy: calls that overlap
// on one device race.
#include <mutex>

#include "common.h"

namespace nosdd {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_lock);
    return g_ptr[device];
}

// One job (tile, rhs) per subdomain and right-hand side, tile-major, for the
// batched block-Thomas solve (the queue that the allocating entry point keeps
// in library-owned memory).
__global__ void noalloc_queue_kernel(int2 *__restrict__ order, int n_tiles, int n_rhs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_tiles * n_rhs) return;
    order[j] = make_int2(j / n_rhs, j - (j / n_rhs) * n_rhs);
}

void launch_noalloc_queue(hipStream_t s, int2 *order, int n_tiles, int n_rhs) {
    const int n = n_tiles * n_rhs;
    hipLaunchKernelGGL(noalloc_queue_kernel, dim3((n + 255) / 256), dim3(256), 0, s, order, n_tiles, n_rhs);
}

}  // namespace nosdd
