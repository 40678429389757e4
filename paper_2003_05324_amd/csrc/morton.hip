// Z-order (Morton) ordering of the locations (the "appropriate ordering" of Section VI).
//
// Key of a point: each coordinate clamped to [0, 1] and quantised to 16 bits,
// q = min(floor(c * 2^16), 2^16 - 1); the bits of q_x go to the even positions and those
// of q_y to the odd positions of a 32-bit key; (longitude, latitude) points in degrees are
// first mapped to ((lon + 180) / 360, (lat + 90) / 180).  Sorting the 64-bit values
// (key << 32) | index ascending gives the stable order by key (ties keep input order).
// The sort is a bitonic network over the padded power-of-two array: stages whose
// partner distance fits in a workgroup run in LDS, the others as global passes.
#include "morton_dev.h"

#include <algorithm>

namespace mpgeo {

namespace {

constexpr int kSortThreads = 512;
constexpr int kSortLocal = 2 * kSortThreads;   // elements held in LDS per workgroup

__global__ void morton_keys_kernel(const double *locs, int64_t n, int64_t n2, int lonlat,
                                   uint64_t *keys) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n2) return;
    if (e >= n) {
        keys[e] = ~0ull;
        return;
    }
    const uint32_t key = morton_key(locs[2 * e], locs[2 * e + 1], lonlat);
    keys[e] = ((uint64_t)key << 32) | (uint64_t)e;
}

// Compare-exchange for one (size, stride) stage over the whole array.
__global__ void bitonic_global_kernel(uint64_t *keys, int64_t n2, int64_t size, int64_t stride) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n2 / 2) return;
    const int64_t lo = (t / stride) * (2 * stride) + (t % stride);
    const int64_t hi = lo + stride;
    const bool ascending = (lo & size) == 0;
    const uint64_t a = keys[lo], b = keys[hi];
    if ((a > b) == ascending) {
        keys[lo] = b;
        keys[hi] = a;
    }
}

// All stages with stride < kSortLocal for one `size` (or, when size == 0, the full
// sort of each kSortLocal block), inside LDS.
__global__ __launch_bounds__(kSortThreads) void bitonic_local_kernel(uint64_t *keys, int64_t size_in) {
    __shared__ uint64_t s[kSortLocal];
    const int64_t base = (int64_t)blockIdx.x * kSortLocal;
    s[threadIdx.x] = keys[base + threadIdx.x];
    s[threadIdx.x + kSortThreads] = keys[base + threadIdx.x + kSortThreads];
    __syncthreads();
    const int64_t first = size_in == 0 ? 2 : size_in;
    const int64_t last = size_in == 0 ? kSortLocal : size_in;
    for (int64_t size = first; size <= last; size *= 2) {
        int64_t stride = size_in == 0 ? size / 2 : kSortLocal / 2;
        for (; stride > 0; stride /= 2) {
            const int t = threadIdx.x;
            const int lo = (int)((t / stride) * (2 * stride) + (t % stride));
            const int hi = lo + (int)stride;
            const bool ascending = ((base + lo) & size) == 0;
            const uint64_t a = s[lo], b = s[hi];
            if ((a > b) == ascending) {
                s[lo] = b;
                s[hi] = a;
            }
            __syncthreads();
        }
    }
    keys[base + threadIdx.x] = s[threadIdx.x];
    keys[base + threadIdx.x + kSortThreads] = s[threadIdx.x + kSortThreads];
}

__global__ void gather_kernel(const double *locs_in, const double *z_in, const uint64_t *keys,
                              int64_t n, double *locs_out, double *z_out, int64_t *perm) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t src = (int64_t)(keys[e] & 0xFFFFFFFFull);
    locs_out[2 * e] = locs_in[2 * src];
    locs_out[2 * e + 1] = locs_in[2 * src + 1];
    if (z_in) z_out[e] = z_in[src];
    perm[e] = src;
}

__global__ void find_nonfinite_kernel(const double *a, int64_t rows, int64_t cols, int64_t ld,
                                      int lower, int *flag) {
    const int64_t total = rows * cols;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % rows, c = e / rows;
        if (lower && r < c) continue;
        bad |= !isfinite(a[r + c * ld]);
    }
    if (bad) *flag = 1;   // every writer stores the same value
}

}  // namespace

void launch_find_nonfinite(const double *a, int64_t rows, int64_t cols, int64_t ld, bool lower,
                           int *flag, hipStream_t stream) {
    const int64_t total = rows * cols;
    if (total <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 2048);
    hipLaunchKernelGGL(find_nonfinite_kernel, dim3(blocks), dim3(256), 0, stream, a, rows, cols, ld,
                       lower ? 1 : 0, flag);
}

// n2 must be a power of two >= max(n, kSortLocal); keys has n2 entries.
void launch_morton_order(const double *locs_in, const double *z_in, int64_t n, bool lonlat,
                         uint64_t *keys, int64_t n2, double *locs_out, double *z_out,
                         int64_t *perm_out, hipStream_t stream) {
    const unsigned kb = (unsigned)((n2 + 255) / 256);
    hipLaunchKernelGGL(morton_keys_kernel, dim3(kb), dim3(256), 0, stream, locs_in, n, n2,
                       lonlat ? 1 : 0, keys);
    const unsigned lb = (unsigned)(n2 / kSortLocal);
    hipLaunchKernelGGL(bitonic_local_kernel, dim3(lb), dim3(kSortThreads), 0, stream, keys,
                       (int64_t)0);
    const unsigned gb = (unsigned)((n2 / 2 + 255) / 256);
    for (int64_t size = 2 * kSortLocal; size <= n2; size *= 2) {
        for (int64_t stride = size / 2; stride >= kSortLocal; stride /= 2)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3(gb), dim3(256), 0, stream, keys, n2,
                               size, stride);
        hipLaunchKernelGGL(bitonic_local_kernel, dim3(lb), dim3(kSortThreads), 0, stream, keys,
                           size);
    }
    const unsigned eb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(gather_kernel, dim3(eb), dim3(256), 0, stream, locs_in, z_in, keys, n,
                       locs_out, z_out, perm_out);
}

}  // namespace mpgeo
