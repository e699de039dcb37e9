// The fixed device array behind cgp_poisson_solve_noalloc, for callers that cannot
// allocate device memory while they run (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  Every buffer such a solve needs beyond the
// mesh's own data and the caller's vectors (the CG vectors, the per-workgroup partial
// sums, the control state, the launch records and the deflation coefficients) is carved
// out of one file-scope device array of CGP_NOALLOC_SCRATCH_BYTES.
//
// Host code never passes the array's name to a kernel: on the host that name is a
// stand-in, not a device address.  cgp_create calls noalloc_init once per device with the
// device current, which looks the array's address up with hipGetSymbolAddress and keeps it
// per device (each GPU holds its own copy, at its own address, until the process ends).
#include <algorithm>
#include <mutex>

#include "cgp_internal.hpp"

namespace cgp {

static __device__ __align__(256) unsigned char scratch[CGP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Writes the records of a no-allocation solve into the scratch array: the instance record,
// the instance index of every stage workgroup and coarse-step workgroup, the coarse-step
// record, and zeros over the deflation coefficients and the coarse partial sums (which
// keep the previous call's values otherwise).
__global__ void k_noalloc_setup(InstDesc *insts, const InstDesc d, int32_t *block_inst, int nblk,
                                int32_t *cblk_inst, int ncb, double *zero, int nzero, CoarseRec *crec,
                                const CoarseRec c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        insts[0] = d;
        if (crec) crec[0] = c;
    }
    if (i < nblk) block_inst[i] = 0;
    if (i < ncb) cblk_inst[i] = 0;
    if (i < nzero) zero[i] = 0.0;
}

}  // namespace

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    CGP_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, "device index beyond the no-allocation table");
    if (g_noalloc_ptr[device]) return;
    void *p = nullptr;
    CGP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    CGP_REQUIRE(p != nullptr, "hipGetSymbolAddress returned a null address for the scratch array");
    g_noalloc_ptr[device] = p;
}

uint8_t *noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    return static_cast<uint8_t *>(g_noalloc_ptr[device]);
}

void launch_noalloc_setup(hipStream_t s, InstDesc *insts, const InstDesc &d, int32_t *block_inst, int nblk,
                          int32_t *cblk_inst, int ncb, double *zero, int nzero, CoarseRec *crec,
                          const CoarseRec &c) {
    const int n = std::max(1, std::max(nblk, std::max(ncb, nzero)));
    hipLaunchKernelGGL(k_noalloc_setup, dim3(blocks_for(n, 256)), dim3(256), 0, s, insts, d, block_inst, nblk,
                       cblk_inst, ncb, zero, nzero, crec, c);
    CGP_HIP(hipGetLastError());
}

}  // namespace cgp
