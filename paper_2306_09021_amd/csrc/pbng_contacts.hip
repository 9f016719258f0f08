// Vertex-vertex proximity detection for dynamic weak constraints (Sec.
// "Collisions": contacts are detected every time step and added as weak
// constraints; the paper leaves the detection itself open).
//
// Candidates are the surface vertices of the workspace (vertices of faces
// with a single incident tet), each with its instance and its connected
// part.  A uniform grid of cell size r is formed by sorting the candidates
// by a 64-bit key (instance, cell x, y, z with 15-bit wrapped cell
// coordinates; wrapping only adds candidates, which the distance test
// removes); the sorts cover only the key bits in use.  Every candidate then looks up the 27 cells around it by binary
// search in the sorted keys and emits each pair (a, b), a < b in caller
// order, of vertices of different parts of one instance within r (not both
// Dirichlet, not coincident).  The pairs are sorted afterwards, so the
// output does not depend on the order of the atomic appends, and each pair
// gets the normal (x_b - x_a) / |x_b - x_a|.
#include <hipcub/hipcub.hpp>

#include "pbng_internal.hpp"

namespace pbng {

namespace {

constexpr int kBlk = 256;

inline int nblocks(int64_t n) { return int((n + kBlk - 1) / kBlk); }

template <class P>
__device__ __forceinline__ void pos_of(const P* x, int g, double* p)
{
    p[0] = double(x[3 * int64_t(g)]);
    p[1] = double(x[3 * int64_t(g) + 1]);
    p[2] = double(x[3 * int64_t(g) + 2]);
}

__device__ __forceinline__ unsigned long long cell_key(int inst, long long cx, long long cy,
                                                       long long cz)
{
    return (static_cast<unsigned long long>(inst) << 45) |
           (static_cast<unsigned long long>(cx & 0x7FFF) << 30) |
           (static_cast<unsigned long long>(cy & 0x7FFF) << 15) |
           static_cast<unsigned long long>(cz & 0x7FFF);
}

__device__ __forceinline__ long long cell_of(double v, double inv_r)
{
    return static_cast<long long>(floor(v * inv_r));
}

template <class P>
__global__ __launch_bounds__(kBlk) void k_keys(const P* x, const ContactCand c, double inv_r,
                                               unsigned long long* keys, int* vals)
{
    const int i = blockIdx.x * kBlk + threadIdx.x;
    if (i >= c.n) return;
    double p[3];
    pos_of(x, c.caller[i], p);
    keys[i] = cell_key(c.inst[i], cell_of(p[0], inv_r), cell_of(p[1], inv_r), cell_of(p[2], inv_r));
    vals[i] = i;
}

__device__ __forceinline__ int lower(const unsigned long long* k, int n, unsigned long long key)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class P>
__global__ __launch_bounds__(kBlk) void k_pairs(const P* x, const ContactCand c, double r,
                                                const unsigned long long* keys, const int* vals,
                                                int max_pairs, int* count, int2* pairs)
{
    const int s = blockIdx.x * kBlk + threadIdx.x;
    if (s >= c.n) return;
    const int i = vals[s];
    const int ga = c.caller[i];
    double pa[3];
    pos_of(x, ga, pa);
    const double inv_r = 1.0 / r;
    const long long cx = cell_of(pa[0], inv_r), cy = cell_of(pa[1], inv_r), cz = cell_of(pa[2], inv_r);
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                const unsigned long long key = cell_key(c.inst[i], cx + dx, cy + dy, cz + dz);
                for (int t = lower(keys, c.n, key); t < c.n && keys[t] == key; ++t) {
                    const int j = vals[t];
                    const int gb = c.caller[j];
                    if (gb <= ga || c.body[j] == c.body[i] || (c.dir[i] && c.dir[j])) continue;
                    double pb[3];
                    pos_of(x, gb, pb);
                    const double d0 = pb[0] - pa[0], d1 = pb[1] - pa[1], d2 = pb[2] - pa[2];
                    const double d = d0 * d0 + d1 * d1 + d2 * d2;
                    if (d > r * r || d == 0.0) continue;
                    const int k = atomicAdd(count, 1);
                    if (k < max_pairs) pairs[k] = int2{ga, gb};
                }
            }
}

// (a, b) as a << vb | b: ascending keys order the pairs by a, then b.
__global__ __launch_bounds__(kBlk) void k_pair_keys(const int2* pairs, int n, int vb, unsigned long long* keys)
{
    const int k = blockIdx.x * kBlk + threadIdx.x;
    if (k >= n) return;
    keys[k] = (static_cast<unsigned long long>(static_cast<unsigned>(pairs[k].x)) << vb) |
              static_cast<unsigned>(pairs[k].y);
}

template <class P>
__global__ __launch_bounds__(kBlk) void k_pair_out(const P* x, const unsigned long long* keys, int n, int vb,
                                                   int* pairs_out, double* normals_out)
{
    const int k = blockIdx.x * kBlk + threadIdx.x;
    if (k >= n) return;
    const int ga = int(keys[k] >> vb), gb = int(keys[k] & ((1ull << vb) - 1));
    double pa[3], pb[3];
    pos_of(x, ga, pa);
    pos_of(x, gb, pb);
    const double d0 = pb[0] - pa[0], d1 = pb[1] - pa[1], d2 = pb[2] - pa[2];
    const double inv = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    pairs_out[2 * k] = ga;
    pairs_out[2 * k + 1] = gb;
    normals_out[3 * k] = d0 * inv;
    normals_out[3 * k + 1] = d1 * inv;
    normals_out[3 * k + 2] = d2 * inv;
}

__global__ __launch_bounds__(kBlk) void k_zero(int* p)
{
    if (threadIdx.x == 0) *p = 0;
}

}  // namespace

template <class P>
hipError_t launch_detect(const P* x, const ContactCand& c, double r, int max_pairs, DetectScratch& w,
                         int* pairs_out, double* normals_out, int* n_found, hipStream_t s)
{
    hipError_t e;
    *n_found = 0;
    if (c.n == 0) return hipSuccess;
    hipLaunchKernelGGL((k_keys<P>), dim3(nblocks(c.n)), dim3(kBlk), 0, s, x, c, 1.0 / r, w.keys_in,
                       w.vals_in);
    size_t tmp = w.tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(w.tmp, tmp, w.keys_in, w.keys_out, w.vals_in, w.vals_out, c.n,
                                           0, 45 + c.inst_bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlk), 0, s, w.count);
    hipLaunchKernelGGL((k_pairs<P>), dim3(nblocks(c.n)), dim3(kBlk), 0, s, x, c, r, w.keys_out,
                       w.vals_out, max_pairs, w.count, w.pairs);
    int h = 0;
    e = hipMemcpyAsync(&h, w.count, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *n_found = h;
    if (h == 0 || h > max_pairs) return hipGetLastError();
    hipLaunchKernelGGL(k_pair_keys, dim3(nblocks(h)), dim3(kBlk), 0, s, w.pairs, h, c.vert_bits, w.pkeys_in);
    tmp = w.tmp_bytes;
    e = hipcub::DeviceRadixSort::SortKeys(w.tmp, tmp, w.pkeys_in, w.pkeys_out, h, 0, 2 * c.vert_bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pair_out<P>), dim3(nblocks(h)), dim3(kBlk), 0, s, x, w.pkeys_out, h, c.vert_bits,
                       pairs_out, normals_out);
    return hipGetLastError();
}

// Temporary bytes hipcub needs for n candidates and max_pairs pairs.
size_t detect_tmp_bytes(int n, int max_pairs)
{
    size_t a = 0, b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (unsigned long long*)nullptr,
                                             (unsigned long long*)nullptr, (int*)nullptr, (int*)nullptr,
                                             n, 0, 64);
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, b, (unsigned long long*)nullptr,
                                            (unsigned long long*)nullptr, max_pairs, 0, 64);
    return a > b ? a : b;
}

template hipError_t launch_detect<float>(const float*, const ContactCand&, double, int, DetectScratch&,
                                         int*, double*, int*, hipStream_t);
template hipError_t launch_detect<double>(const double*, const ContactCand&, double, int, DetectScratch&,
                                          int*, double*, int*, hipStream_t);

}  // namespace pbng
