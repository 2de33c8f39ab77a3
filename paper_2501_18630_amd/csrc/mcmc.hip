// Kernel-agnostic MCMC step of Sec. 3.4.
//
// Noise (Optimization paragraph): mu += lambda_eps lr B(o; b') eta, with the
// Beta kernel B(o; b') = (1 - o)^(4 e^b') and eta = R diag(s) z a sample of
// N(0, Sigma) for the caller's standard normals z.
//
// Relocation (Densification paragraph and its appendix): a primitive with
// o <= tau is dead.  Each dead primitive i copies a live primitive j drawn in
// proportion to opacity from the caller's uniform 32-bit u_i: with weights
// w_j = floor(o_j 2^24) (exact integers, so the draw is an exact decision)
// and inclusive prefix sums P_j, i takes the first j with P_j > t_i,
// t_i = floor(u_i W / 2^32).  A live primitive drawn N - 1 times ends with N
// copies, all of opacity o' = 1 - (1 - o)^(1/N); nothing else is adjusted.
//
// Pipeline: weights and per-block sums -> scan of the block sums -> prefix
// sums -> draw + copy counts -> new opacities -> copies.  Everything is
// integer except o', evaluated in FP64 as -expm1(log1p(-o) / N).
#include "dbs_internal.h"

namespace dbs {

namespace {

constexpr int kMcmcBlock = 1024;  // elements per block of the prefix pipeline (256 threads x 4)

__device__ __forceinline__ uint32_t opacity_weight(float o, float tau)
{
    return o <= tau ? 0u : (uint32_t)(o * 16777216.0f);  // o * 2^24 is exact; truncation = floor
}

__device__ __forceinline__ uint64_t block_inclusive_scan_u64(uint64_t v, uint64_t *s_tmp /*[5]*/, uint64_t *total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) s_tmp[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = 0;
        for (int k = 0; k < 4; ++k) {
            const uint64_t c = s_tmp[k];
            s_tmp[k] = acc;
            acc += c;
        }
        s_tmp[4] = acc;
    }
    __syncthreads();
    const uint64_t r = s_tmp[w] + x;
    if (total) *total = s_tmp[4];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void weight_sums_kernel(const float *o, int64_t n, float tau, uint64_t *bsum)
{
    __shared__ uint64_t s_tmp[5];
    const int64_t base = (int64_t)blockIdx.x * kMcmcBlock + threadIdx.x * 4;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < n) acc += opacity_weight(o[base + k], tau);
    uint64_t tot;
    block_inclusive_scan_u64(acc, s_tmp, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block sums in place (one workgroup); bsum[nb] = W.
__global__ __launch_bounds__(256) void scan_block_sums_kernel(uint64_t *bsum, int64_t nb)
{
    __shared__ uint64_t s_tmp[5];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const uint64_t v = b < nb ? bsum[b] : 0;
        uint64_t tot;
        const uint64_t inc = block_inclusive_scan_u64(v, s_tmp, &tot);
        if (b < nb) bsum[b] = s_carry + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = s_carry;
}

__global__ __launch_bounds__(256) void weight_prefix_kernel(const float *o, int64_t n, float tau, const uint64_t *bsum,
                                                            uint64_t *prefix, uint32_t *count)
{
    __shared__ uint64_t s_tmp[5];
    const int64_t base = (int64_t)blockIdx.x * kMcmcBlock + threadIdx.x * 4;
    uint32_t w[4];
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = base + k < n ? opacity_weight(o[base + k], tau) : 0u;
        acc += w[k];
    }
    uint64_t run = block_inclusive_scan_u64(acc, s_tmp, nullptr) - acc + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) {
            run += w[k];
            prefix[base + k] = run;  // inclusive
            count[base + k] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void draw_kernel(const float *o, int64_t n, float tau, const uint32_t *rand,
                                                   const uint64_t *prefix, const uint64_t *total_p, uint32_t *target,
                                                   uint32_t *count, int32_t *n_relocated)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = *total_p;
    bool moved = false;
    if (i < n) {
        uint32_t tgt = 0xffffffffu;
        if (o[i] <= tau && total > 0) {
            const uint64_t u = rand[i], hi = total >> 32, lo = total & 0xffffffffull;
            const uint64_t t = u * hi + ((u * lo) >> 32);  // floor(u W / 2^32)
            int64_t a = 0, b = n - 1;                      // first j with prefix[j] > t
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if (prefix[mid] > t) b = mid; else a = mid + 1;
            }
            tgt = (uint32_t)a;
            atomicAdd(&count[a], 1u);
            moved = true;
        }
        target[i] = tgt;
    }
    if (n_relocated) {
        const uint64_t bal = __ballot(moved);
        if ((threadIdx.x & (kWave - 1)) == 0 && bal) atomicAdd(n_relocated, (int32_t)__popcll(bal));
    }
}

__global__ __launch_bounds__(256) void new_opacity_kernel(const float *o, int64_t n, const uint32_t *count,
                                                          float *onew)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && count[i] > 0) onew[i] = (float)(-expm1(log1p(-(double)o[i]) / (double)(count[i] + 1)));
}

__global__ __launch_bounds__(256) void relocate_kernel(SplatMut p, const uint32_t *target, const uint32_t *count,
                                                       const float *onew)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const uint32_t j = target[i];
    if (j != 0xffffffffu) {  // dead: becomes a copy of j
        for (int k = 0; k < 3; ++k) {
            p.means[3 * i + k] = p.means[3 * (int64_t)j + k];
            p.scales[3 * i + k] = p.scales[3 * (int64_t)j + k];
            p.diffuse[3 * i + k] = p.diffuse[3 * (int64_t)j + k];
        }
        for (int k = 0; k < 4; ++k) p.quats[4 * i + k] = p.quats[4 * (int64_t)j + k];
        p.betas[i] = p.betas[j];
        p.opacities[i] = onew[j];
        for (int l = 0; l < p.m; ++l) {
            const int64_t di = i * p.m + l, dj = (int64_t)j * p.m + l;
            p.lobe_angles[2 * di] = p.lobe_angles[2 * dj];
            p.lobe_angles[2 * di + 1] = p.lobe_angles[2 * dj + 1];
            for (int c = 0; c < 3; ++c) p.lobe_colors[3 * di + c] = p.lobe_colors[3 * dj + c];
            p.lobe_betas[di] = p.lobe_betas[dj];
        }
    } else if (count[i] > 0) {
        p.opacities[i] = onew[i];
    }
}

__global__ void zero_i32_kernel(int32_t *p) { *p = 0; }

__global__ __launch_bounds__(256) void noise_kernel(SplatMut p, const float *z, float amp, float beta_noise)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n) return;
    const float o = p.opacities[i];
    const float one_m = 1.0f - o;
    const float bk = one_m > 0.0f ? exp2f(beta_noise * log2f(one_m)) : 0.0f;  // (1 - o)^(4 e^b')
    float q0 = p.quats[4 * i], q1 = p.quats[4 * i + 1], q2 = p.quats[4 * i + 2], q3 = p.quats[4 * i + 3];
    const float inv = rsqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    q0 *= inv; q1 *= inv; q2 *= inv; q3 *= inv;
    const float R[9] = {1.f - 2.f * (q2 * q2 + q3 * q3), 2.f * (q1 * q2 - q0 * q3), 2.f * (q1 * q3 + q0 * q2),
                        2.f * (q1 * q2 + q0 * q3), 1.f - 2.f * (q1 * q1 + q3 * q3), 2.f * (q2 * q3 - q0 * q1),
                        2.f * (q1 * q3 - q0 * q2), 2.f * (q2 * q3 + q0 * q1), 1.f - 2.f * (q1 * q1 + q2 * q2)};
    const float sz[3] = {p.scales[3 * i] * z[3 * i], p.scales[3 * i + 1] * z[3 * i + 1],
                         p.scales[3 * i + 2] * z[3 * i + 2]};
    const float f = amp * bk;
    for (int r = 0; r < 3; ++r) p.means[3 * i + r] += f * (R[3 * r] * sz[0] + R[3 * r + 1] * sz[1] + R[3 * r + 2] * sz[2]);
}

}  // namespace

McmcLayout mcmc_layout(int64_t n)
{
    McmcLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) & ~(size_t)255;
        return at;
    };
    const int64_t nb = ceil_div(n > 0 ? n : 1, kMcmcBlock);
    L.nblocks = nb;
    L.bsum = take((size_t)(nb + 1) * 8);
    L.prefix = take((size_t)(n > 0 ? n : 1) * 8);
    L.count = take((size_t)(n > 0 ? n : 1) * 4);
    L.target = take((size_t)(n > 0 ? n : 1) * 4);
    L.onew = take((size_t)(n > 0 ? n : 1) * 4);
    L.total = o;
    return L;
}

hipError_t launch_mcmc_relocate(const SplatMut &p, float tau, const uint32_t *rand, void *work, int32_t *n_relocated,
                                hipStream_t s)
{
    if (n_relocated) zero_i32_kernel<<<1, 1, 0, s>>>(n_relocated);
    if (p.n <= 0) return hipGetLastError();
    const McmcLayout L = mcmc_layout(p.n);
    char *w = (char *)work;
    uint64_t *bsum = (uint64_t *)(w + L.bsum), *prefix = (uint64_t *)(w + L.prefix);
    uint32_t *count = (uint32_t *)(w + L.count), *target = (uint32_t *)(w + L.target);
    float *onew = (float *)(w + L.onew);
    const unsigned nb = (unsigned)L.nblocks, gt = (unsigned)ceil_div(p.n, 256);
    weight_sums_kernel<<<nb, 256, 0, s>>>(p.opacities, p.n, tau, bsum);
    scan_block_sums_kernel<<<1, 256, 0, s>>>(bsum, L.nblocks);
    weight_prefix_kernel<<<nb, 256, 0, s>>>(p.opacities, p.n, tau, bsum, prefix, count);
    draw_kernel<<<gt, 256, 0, s>>>(p.opacities, p.n, tau, rand, prefix, bsum + L.nblocks, target, count, n_relocated);
    new_opacity_kernel<<<gt, 256, 0, s>>>(p.opacities, p.n, count, onew);
    relocate_kernel<<<gt, 256, 0, s>>>(p, target, count, onew);
    return hipGetLastError();
}

hipError_t launch_mcmc_noise(const SplatMut &p, const float *z, float lr, float lambda_eps, float b_prime,
                             hipStream_t s)
{
    if (p.n <= 0) return hipSuccess;
    const float beta_noise = (float)(4.0 * exp((double)b_prime));
    noise_kernel<<<(unsigned)ceil_div(p.n, 256), 256, 0, s>>>(p, z, lambda_eps * lr, beta_noise);
    return hipGetLastError();
}

}  // namespace dbs
