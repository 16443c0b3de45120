// Multi-stream serving kernel: one launch runs the next frame of many camera
// streams -- mixed resolutions, GMM and PBAS together -- over a flat list of
// tiles.  Each workgroup walks the list with a grid stride, finds a tile's entry
// by binary search over the tile prefix sums and runs the same per-pixel (GMM)
// or per-tile (PBAS) device code as the per-frame kernels, so a stream's result
// does not depend on what it is batched with.
#include "device_common.h"
#include "fgs_internal.h"
#include "gmm_device.h"
#include "pbas_device.h"

namespace fgs {

namespace {

template <int KG, int NP, bool NT>
__global__ __launch_bounds__(256) void serve_kernel(const ServeEntry* __restrict__ entries,
                                                    const int32_t* __restrict__ prefix, int n) {
    __shared__ pbas::PbasLds<NP> sh;
    const int total = prefix[n];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = n;  // prefix[lo] <= w < prefix[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= w) lo = mid;
            else hi = mid;
        }
        const ServeEntry& e = entries[lo];
        const int local = w - prefix[lo];
        if (e.algo == FGS_GMM) {
            const int p = local * 256 + (int)threadIdx.x;
            if (p < e.g.npix) gmm_pixel<KG, KG, NT>(e.g, p);
        } else if (e.fill) {
            const int p = local * 256 + (int)threadIdx.x;
            if (p < e.p.npix) pbas::fill_pixel(e.p, p);
        } else {
            pbas::pbas_tile<NP, 2, NT>(e.p, local % e.tiles_x, local / e.tiles_x, sh);  // any N <= NP
        }
        __syncthreads();  // the next tile reuses the LDS
    }
}

template <int KG, int NP>
void launch(const ServeEntry* e, const int32_t* prefix, int n, int grid, bool nt, hipStream_t s) {
    if (nt) hipLaunchKernelGGL((serve_kernel<KG, NP, true>), dim3(grid), dim3(256), 0, s, e, prefix, n);
    else hipLaunchKernelGGL((serve_kernel<KG, NP, false>), dim3(grid), dim3(256), 0, s, e, prefix, n);
}

}  // namespace

int serve_pbas_nmax(int N) { return N <= 24 ? 24 : (N <= 40 ? 40 : 0); }

hipError_t serve_launch(const ServeEntry* entries, const int32_t* prefix, int n, int total_tiles,
                        int gmm_K, int pbas_nmax, bool streaming, hipStream_t s) {
    if (n <= 0 || total_tiles <= 0) return hipSuccess;
    const int grid = total_tiles < 256 * 8 ? total_tiles : 256 * 8;  // 8 workgroups per CU
    const int key = gmm_K * 100 + pbas_nmax;
    switch (key) {
        case 324: launch<3, 24>(entries, prefix, n, grid, streaming, s); break;
        case 340: launch<3, 40>(entries, prefix, n, grid, streaming, s); break;
        case 524: launch<5, 24>(entries, prefix, n, grid, streaming, s); break;
        case 540: launch<5, 40>(entries, prefix, n, grid, streaming, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fgs
