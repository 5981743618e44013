// Lattice-independent kernels: per-lattice reduction of the per-tile
// diagnostics in a fixed order, and a plain copy kernel used to calibrate
// hardware traffic counters.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_shared.hpp"

namespace lbm {

// One block per lattice; each thread folds a strided subset of the lattice's
// tiles, then a fixed-shape tree combines the threads: the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void finalize_diag_kernel(const DiagPartial* partial, const LatticeRec* recs,
                                                            const unsigned* status, DiagOut* out) {
    const LatticeRec& R = recs[blockIdx.x];
    __shared__ double sh[7][256];
    __shared__ unsigned shs[256];
    double m = 0, mx = 0, my = 0, mz = 0, u2 = 0, mn = 1e300, mxv = -1e300;
    unsigned st = 0;
    for (int t = R.tile_begin + threadIdx.x; t < R.tile_end; t += 256) {
        const DiagPartial p = partial[t];
        m += p.mass; mx += p.momx; my += p.momy; mz += p.momz;
        u2 = fmax(u2, p.umax2); mn = fmin(mn, p.mumin); mxv = fmax(mxv, p.mumax);
        st |= p.status;
    }
    const int i = threadIdx.x;
    sh[0][i] = m; sh[1][i] = mx; sh[2][i] = my; sh[3][i] = mz; sh[4][i] = u2; sh[5][i] = mn; sh[6][i] = mxv;
    shs[i] = st;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w) {
            sh[0][i] += sh[0][i + w]; sh[1][i] += sh[1][i + w]; sh[2][i] += sh[2][i + w]; sh[3][i] += sh[3][i + w];
            sh[4][i] = fmax(sh[4][i], sh[4][i + w]);
            sh[5][i] = fmin(sh[5][i], sh[5][i + w]);
            sh[6][i] = fmax(sh[6][i], sh[6][i + w]);
            shs[i] |= shs[i + w];
        }
        __syncthreads();
    }
    if (i == 0) {
        DiagOut o;
        o.mass = sh[0][0] + (double)R.nnodes * R.rho_ref;
        o.momx = sh[1][0]; o.momy = sh[2][0]; o.momz = sh[3][0];
        o.umax = sqrt(sh[4][0]);
        o.mumin = sh[5][0]; o.mumax = sh[6][0];
        o.status = shs[0] | status[blockIdx.x];
        o.pad = 0;
        out[blockIdx.x] = o;
    }
}

// Plain copy: one 16-byte vector per thread, the grid covering the buffer once
// and no grid-stride loop, so the work groups in flight at any time touch one
// compact address window (a grid-stride loop spreads them over the whole buffer
// and streams about a quarter slower); non-temporal stores like the step
// kernels' population stores.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(uint4* __restrict__ dst_, const uint4* __restrict__ src_,
                                                   size_t n16) {
    v4u* __restrict__ dst = reinterpret_cast<v4u*>(dst_);
    const v4u* __restrict__ src = reinterpret_cast<const v4u*>(src_);
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(src[i], dst + i);
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_finalize(const DiagPartial* partial, const LatticeRec* recs, const unsigned* status,
                           DiagOut* out, int nlat, hipStream_t s) {
    hipLaunchKernelGGL(finalize_diag_kernel, dim3(nlat), dim3(256), 0, s, partial, recs, status, out);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    constexpr size_t kMaxBlocks = 1u << 30;                  // per launch
    for (size_t done = 0; done < n16;) {
        const size_t n = std::min(n16 - done, kMaxBlocks * 256);
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (uint4*)dst + done, (const uint4*)src + done, n);
        done += n;
    }
    const size_t rest = bytes - n16 * 16;
    if (rest) {
        hipError_t e = hipMemcpyAsync((char*)dst + n16 * 16, (const char*)src + n16 * 16, rest,
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace lbm
