// Batched evaluation of the AMI solution on gfx950 (Burke & LeBlanc,
// arXiv 2311.17189, Sec. 2.3): for N_E energy rows and N_F external-frequency
// rows, out[f][s] = sum_t A_t * FT_t(E_s) * R_t(E_s, w_f)  (Eq. (6)).
//
// Mapping: one lane per energy sample, 64-lane wavefronts, blocks of 64..256
// lanes.  Per sample the kernel
//   1. loads the energies (or momenta, computing E_j = 2t(cos Kx + cos Ky) + mu
//      with K_j = sum_l alpha_jl k_l, Sec. 5.2) into registers;
//   2. evaluates every distinct Fermi/Bose leaf once into LDS (column per lane);
//   3. sums the Fermi-tree products of each group of terms that share their
//      denominators: FT_g = sum_{t in g} s_t prod_leaves; FT_g does not depend
//      on the external frequency (Sec. 2.2, Sec. 2.3) and is kept in LDS;
//   4. per frequency row: distinct denominators -> complex reciprocals in LDS,
//      R_g = product over the group's denominators, out = sum_g FT_g * R_g.
// Integer coefficient tables are read with wave-uniform addresses (scalar
// loads); the only per-lane memory traffic is the sample input and the output.
// Row sums (Monte-Carlo averages of Sec. 2.3) are reduced per block with a
// fixed shuffle tree and then across blocks in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "ami_internal.hpp"

namespace ami {

namespace {

inline AmiStatus hip_fail(hipError_t e, const char *what) {
    return fail(AMI_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct FwdParams {
    // tables
    const double *leaf_coef;
    const double *leaf_sigma;
    const double *den_coef;
    const int32_t *group_dens;
    const int32_t *group_start;
    const double *term_sign;
    const int32_t *term_leaf;
    const double *line_alpha;
    int n_eps, n_ext, n_int, n_g, n_freq;
    int L, D, G, dpt;
    int region_a;            // LDS slots (per lane) before the FT region: max(L, 2D)
    // energy input
    const double *energies;
    int64_t stride_s, stride_i;
    // momentum input
    const double *k;
    int64_t stride_k;
    double q[2 * kMaxExt];
    double hop_t, mu;
    // frequencies, parameters, outputs
    const double *ext_freqs;
    int n_f;
    double beta, e_reg;
    int64_t n_e;
    double *out;
    double *partial;          // [gridDim.x][n_f][2] or NULL
};

// f_sigma(y) = 1/(sigma e^y + 1).  The Bose-type form -1/expm1(y) keeps full
// relative precision next to its removable pole at y = 0.
__device__ __forceinline__ double leaf_fn(double sigma, double y) {
    if (sigma > 0.0) return 1.0 / (1.0 + exp(y));
    return -1.0 / expm1(y);
}

template <int MAXE, bool HUB>
__global__ __launch_bounds__(256) void ami_fwd_kernel(FwdParams p) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x;
    const int B = blockDim.x;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * B + tid;
    const bool active = s < p.n_e;
    const int64_t sc = active ? s : (p.n_e - 1);

    double E[MAXE];
#pragma unroll
    for (int i = 0; i < MAXE; ++i) E[i] = 0.0;

    if constexpr (HUB) {
        // momenta of the summed slots in registers; external momenta are kernel arguments
        double kx[kMaxInt], ky[kMaxInt];
        const double *krow = p.k + sc * p.stride_k;
#pragma unroll
        for (int l = 0; l < kMaxInt; ++l) {
            kx[l] = 0.0;
            ky[l] = 0.0;
            if (l < p.n_int) {
                kx[l] = krow[2 * l];
                ky[l] = krow[2 * l + 1];
            }
        }
#pragma unroll
        for (int j = 0; j < MAXE; ++j) {
            if (j < p.n_g) {
                // K_j = sum_l alpha_jl k_l (Sec. 5.2), E_j = -eps(K_j) = 2t(cos Kx + cos Ky) + mu
                const double *a = p.line_alpha + j * p.n_freq;
                double Kx = 0.0, Ky = 0.0;
#pragma unroll
                for (int l = 0; l < kMaxInt; ++l) {
                    if (l < p.n_int) {
                        Kx = fma(a[l], kx[l], Kx);
                        Ky = fma(a[l], ky[l], Ky);
                    }
                }
#pragma unroll
                for (int x = 0; x < kMaxExt; ++x) {
                    if (x < p.n_ext) {
                        Kx = fma(a[p.n_int + x], p.q[2 * x], Kx);
                        Ky = fma(a[p.n_int + x], p.q[2 * x + 1], Ky);
                    }
                }
                E[j] = fma(2.0 * p.hop_t, cos(Kx) + cos(Ky), p.mu);
            }
        }
    } else {
        const double *erow = p.energies + sc * p.stride_s;
#pragma unroll
        for (int i = 0; i < MAXE; ++i)
            if (i < p.n_eps) E[i] = erow[i * p.stride_i];
    }

    // 2. distinct leaves -> LDS
    for (int l = 0; l < p.L; ++l) {
        const double *c = p.leaf_coef + l * p.n_eps;
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < MAXE; ++i)
            if (i < p.n_eps) x = fma(c[i], E[i], x);
        const double sg = p.leaf_sigma[l];
        if (sg < 0.0) x += p.e_reg;
        sm[l * B + tid] = leaf_fn(sg, p.beta * x);
    }

    // 3. Fermi-tree sums per group of equal denominators -> LDS
    double *ftcol = sm + p.region_a * B;
    for (int g = 0; g < p.G; ++g) {
        const int t0 = p.group_start[g], t1 = p.group_start[g + 1];
        double ft = 0.0;
        for (int t = t0; t < t1; ++t) {
            double prod = p.term_sign[t];
            const int32_t *li = p.term_leaf + t * p.n_int;
            for (int j = 0; j < p.n_int; ++j) prod *= sm[li[j] * B + tid];
            ft += prod;
        }
        ftcol[g * B + tid] = ft;
    }

    // 4. per frequency row
    double *red = sm + (p.region_a + p.G) * B;     // 2 doubles per wave
    const int wave = tid >> 6, lane = tid & 63, nwaves = (B + 63) >> 6;
    const int ncoef = p.n_eps + p.n_ext;
    for (int f = 0; f < p.n_f; ++f) {
        double wre[kMaxExt], wim[kMaxExt];
#pragma unroll
        for (int x = 0; x < kMaxExt; ++x) {
            wre[x] = 0.0;
            wim[x] = 0.0;
            if (x < p.n_ext) {
                wre[x] = p.ext_freqs[2 * (f * p.n_ext + x)];
                wim[x] = p.ext_freqs[2 * (f * p.n_ext + x) + 1];
            }
        }
        for (int r = 0; r < p.D; ++r) {
            const double *c = p.den_coef + r * ncoef;
            double dre = 0.0, dim = 0.0;
#pragma unroll
            for (int i = 0; i < MAXE; ++i)
                if (i < p.n_eps) dre = fma(c[i], E[i], dre);
#pragma unroll
            for (int x = 0; x < kMaxExt; ++x) {
                if (x < p.n_ext) {
                    dre = fma(c[p.n_eps + x], wre[x], dre);
                    dim = fma(c[p.n_eps + x], wim[x], dim);
                }
            }
            const double inv = 1.0 / fma(dre, dre, dim * dim);
            sm[(2 * r) * B + tid] = dre * inv;
            sm[(2 * r + 1) * B + tid] = -dim * inv;
        }
        double acc_re = 0.0, acc_im = 0.0;
        for (int g = 0; g < p.G; ++g) {
            double rr = 1.0, ri = 0.0;
            const int32_t *gd = p.group_dens + g * p.dpt;
            for (int k = 0; k < p.dpt; ++k) {
                const int d = gd[k];
                const double xr = sm[(2 * d) * B + tid], xi = sm[(2 * d + 1) * B + tid];
                const double nr = fma(rr, xr, -ri * xi);
                ri = fma(rr, xi, ri * xr);
                rr = nr;
            }
            const double ft = ftcol[g * B + tid];
            acc_re = fma(ft, rr, acc_re);
            acc_im = fma(ft, ri, acc_im);
        }
        if (active && p.out) {
            double2 v;
            v.x = acc_re;
            v.y = acc_im;
            reinterpret_cast<double2 *>(p.out)[static_cast<int64_t>(f) * p.n_e + s] = v;
        }
        if (p.partial) {
            double vr = active ? acc_re : 0.0, vi = active ? acc_im : 0.0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                vr += __shfl_xor(vr, off, 64);
                vi += __shfl_xor(vi, off, 64);
            }
            if (lane == 0) {
                red[2 * wave] = vr;
                red[2 * wave + 1] = vi;
            }
            __syncthreads();
            if (tid == 0) {
                double sr = 0.0, si = 0.0;
                for (int w = 0; w < nwaves; ++w) {
                    sr += red[2 * w];
                    si += red[2 * w + 1];
                }
                p.partial[(static_cast<int64_t>(blockIdx.x) * p.n_f + f) * 2] = sr;
                p.partial[(static_cast<int64_t>(blockIdx.x) * p.n_f + f) * 2 + 1] = si;
            }
            __syncthreads();
        }
    }
}

// out_sum[f] = sum over blocks of partial[b][f], in a fixed order.
__global__ __launch_bounds__(256) void ami_rowsum_kernel(const double *partial, int64_t nblocks, int n_f,
                                                         double *out_sum) {
    __shared__ double sr[256], si[256];
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int64_t b = tid; b < nblocks; b += 256) {
        ar += partial[(b * n_f + f) * 2];
        ai += partial[(b * n_f + f) * 2 + 1];
    }
    sr[tid] = ar;
    si[tid] = ai;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) {
            sr[tid] += sr[tid + w];
            si[tid] += si[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out_sum[2 * f] = sr[0];
        out_sum[2 * f + 1] = si[0];
    }
}

__global__ void ami_fill_kernel(double *p, int64_t n, double v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Upload (once per device) the flattened tables of a handle.
AmiStatus upload(AmiTerms *t, DeviceTables **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(t->dev_mu);
    for (auto &d : t->dev)
        if (d.device == dev) {
            *out = &d;
            return AMI_OK;
        }
    const Tables &tb = t->tab;
    struct Piece {
        const void *src;
        size_t bytes;
        size_t off;
    };
    Piece pieces[8] = {
        {tb.leaf_coef.data(), tb.leaf_coef.size() * sizeof(double), 0},
        {tb.leaf_sigma.data(), tb.leaf_sigma.size() * sizeof(double), 0},
        {tb.den_coef.data(), tb.den_coef.size() * sizeof(double), 0},
        {tb.group_dens.data(), tb.group_dens.size() * sizeof(int32_t), 0},
        {tb.group_start.data(), tb.group_start.size() * sizeof(int32_t), 0},
        {tb.term_sign.data(), tb.term_sign.size() * sizeof(double), 0},
        {tb.term_leaf.data(), tb.term_leaf.size() * sizeof(int32_t), 0},
        {tb.line_alpha.data(), tb.line_alpha.size() * sizeof(double), 0},
    };
    size_t total = 0;
    for (auto &pc : pieces) {
        pc.off = total;
        total += align256(std::max<size_t>(pc.bytes, 8));
    }
    std::vector<unsigned char> host(total, 0);
    for (auto &pc : pieces)
        if (pc.bytes) std::memcpy(host.data() + pc.off, pc.src, pc.bytes);
    void *blob = nullptr;
    e = hipMalloc(&blob, total);
    if (e != hipSuccess) return fail(AMI_E_OOM, std::string("hipMalloc of tables: ") + hipGetErrorString(e));
    e = hipMemcpy(blob, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(blob);
        return hip_fail(e, "hipMemcpy of tables");
    }
    DeviceTables d;
    d.device = dev;
    d.blob = blob;
    auto at = [&](int i) { return static_cast<unsigned char *>(blob) + pieces[i].off; };
    d.leaf_coef = reinterpret_cast<const double *>(at(0));
    d.leaf_sigma = reinterpret_cast<const double *>(at(1));
    d.den_coef = reinterpret_cast<const double *>(at(2));
    d.group_dens = reinterpret_cast<const int32_t *>(at(3));
    d.group_start = reinterpret_cast<const int32_t *>(at(4));
    d.term_sign = reinterpret_cast<const double *>(at(5));
    d.term_leaf = reinterpret_cast<const int32_t *>(at(6));
    d.line_alpha = reinterpret_cast<const double *>(at(7));
    t->dev.push_back(d);
    *out = &t->dev.back();
    return AMI_OK;
}

struct LaunchShape {
    int block = 256;
    size_t lds = 0;
    int region_a = 0;
};

AmiStatus pick_shape(const AmiTerms *t, LaunchShape &ls) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    const Tables &tb = t->tab;
    ls.region_a = std::max(tb.L, 2 * tb.D);
    const size_t per_lane = static_cast<size_t>(ls.region_a + tb.G) * sizeof(double);
    // prefer 256 lanes while one block stays within a quarter of the CU's LDS
    const int blocks[3] = {256, 128, 64};
    for (int b : blocks) {
        const size_t lds = per_lane * b + 2 * sizeof(double) * (b / 64);
        if (lds <= static_cast<size_t>(max_lds) && (lds <= 40 * 1024 || b == 64)) {
            ls.block = b;
            ls.lds = lds;
            return AMI_OK;
        }
    }
    return fail(AMI_E_UNSUPPORTED, "solution too large for the LDS-resident evaluator (" +
                                       std::to_string(per_lane) + " B per sample)");
}

AmiStatus launch_forward(AmiTerms *t, bool hub, FwdParams &p, double *out_sum, hipStream_t stream) {
    DeviceTables *dt = nullptr;
    AmiStatus st = upload(t, &dt);
    if (st != AMI_OK) return st;
    const Tables &tb = t->tab;
    p.leaf_coef = dt->leaf_coef;
    p.leaf_sigma = dt->leaf_sigma;
    p.den_coef = dt->den_coef;
    p.group_dens = dt->group_dens;
    p.group_start = dt->group_start;
    p.term_sign = dt->term_sign;
    p.term_leaf = dt->term_leaf;
    p.line_alpha = dt->line_alpha;
    p.n_eps = t->n_eps;
    p.n_ext = t->n_ext;
    p.n_int = t->n_int;
    p.n_g = t->n_g;
    p.n_freq = t->n_freq;
    p.L = tb.L;
    p.D = tb.D;
    p.G = tb.G;
    p.dpt = tb.dpt;
    if (p.n_e == 0) {
        if (out_sum) {
            hipLaunchKernelGGL(ami_fill_kernel, dim3((2 * p.n_f + 255) / 256), dim3(256), 0, stream, out_sum,
                               static_cast<int64_t>(2 * p.n_f), 0.0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "fill launch");
        }
        return AMI_OK;
    }
    LaunchShape ls;
    st = pick_shape(t, ls);
    if (st != AMI_OK) return st;
    p.region_a = ls.region_a;
    const int64_t nblocks = (p.n_e + ls.block - 1) / ls.block;
    if (nblocks > 0x7fffffffLL) return fail(AMI_E_ARG, "n_e too large");
    double *partial = nullptr;
    hipError_t e;
    if (out_sum) {
        e = hipMallocAsync(reinterpret_cast<void **>(&partial), static_cast<size_t>(nblocks) * p.n_f * 2 * sizeof(double),
                           stream);
        if (e != hipSuccess) return fail(AMI_E_OOM, std::string("workspace: ") + hipGetErrorString(e));
    }
    p.partial = partial;
    const int maxe = t->n_eps <= 4 ? 4 : (t->n_eps <= 8 ? 8 : 16);
    const dim3 grid(static_cast<unsigned>(nblocks)), block(ls.block);
#define AMI_LAUNCH(ME, H) hipLaunchKernelGGL((ami_fwd_kernel<ME, H>), grid, block, ls.lds, stream, p)
    if (hub) {
        if (maxe == 4) AMI_LAUNCH(4, true);
        else if (maxe == 8) AMI_LAUNCH(8, true);
        else AMI_LAUNCH(16, true);
    } else {
        if (maxe == 4) AMI_LAUNCH(4, false);
        else if (maxe == 8) AMI_LAUNCH(8, false);
        else AMI_LAUNCH(16, false);
    }
#undef AMI_LAUNCH
    e = hipGetLastError();
    if (e != hipSuccess) {
        if (partial) (void)hipFreeAsync(partial, stream);
        return hip_fail(e, "forward launch");
    }
    if (out_sum) {
        hipLaunchKernelGGL(ami_rowsum_kernel, dim3(p.n_f), dim3(256), 0, stream, partial, nblocks, p.n_f, out_sum);
        e = hipGetLastError();
        (void)hipFreeAsync(partial, stream);
        if (e != hipSuccess) return hip_fail(e, "row-sum launch");
    }
    return AMI_OK;
}

AmiStatus check_common(const AmiTerms *t, int64_t n_e, const double *ext_freqs, int64_t n_f, double beta,
                       const double *out, const double *out_sum) {
    if (!t) return fail(AMI_E_ARG, "terms is NULL");
    if (n_e < 0) return fail(AMI_E_ARG, "n_e < 0");
    if (n_f < 1 || n_f > (1 << 24)) return fail(AMI_E_ARG, "n_f must be in 1..2^24");
    if (!ext_freqs && t->n_ext > 0) return fail(AMI_E_ARG, "ext_freqs is NULL");
    if (!(beta > 0.0)) return fail(AMI_E_ARG, "beta must be > 0");
    if (!out && !out_sum) return fail(AMI_E_ARG, "out and out_sum are both NULL");
    if (t->n_eps > kMaxEpsDev) return fail(AMI_E_UNSUPPORTED, "more than 16 energy placeholders");
    if (t->n_ext > kMaxExt) return fail(AMI_E_UNSUPPORTED, "more than 4 external frequency slots");
    return AMI_OK;
}

}  // namespace

}  // namespace ami

extern "C" {

AmiStatus amiTermsUpload(AmiTerms *t) {
    ami::clear_error();
    if (!t) return ami::fail(AMI_E_ARG, "terms is NULL");
    ami::DeviceTables *dt = nullptr;
    return ami::upload(t, &dt);
}

void amiFree(AmiTerms *t) {
    if (!t) return;
    int cur = 0;
    bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (auto &d : t->dev) {
        if (d.blob) {
            if (hipSetDevice(d.device) == hipSuccess) (void)hipFree(d.blob);
        }
    }
    if (have_cur) (void)hipSetDevice(cur);
    delete t;
}

AmiStatus amiEvaluate(AmiTerms *t, const double *energies, int64_t n_e, int64_t stride_s, int64_t stride_i,
                      const double *ext_freqs, int64_t n_f, double beta, double e_reg, double *out,
                      double *out_sum, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta, out, out_sum);
    if (st != AMI_OK) return st;
    if (n_e > 0 && !energies) return fail(AMI_E_ARG, "energies is NULL");
    if (n_e > 0 && (stride_i < 1 || stride_s < 1)) return fail(AMI_E_ARG, "strides must be >= 1");
    FwdParams p;
    std::memset(&p, 0, sizeof(p));
    p.energies = energies;
    p.stride_s = stride_s;
    p.stride_i = stride_i;
    p.ext_freqs = ext_freqs;
    p.n_f = static_cast<int>(n_f);
    p.beta = beta;
    p.e_reg = e_reg;
    p.n_e = n_e;
    p.out = out;
    return launch_forward(t, false, p, out_sum, static_cast<hipStream_t>(hip_stream));
}

AmiStatus amiEvaluateHubbard(AmiTerms *t, const double *k, int64_t n_e, int64_t stride_k, const double *q,
                             double hop_t, double mu, const double *ext_freqs, int64_t n_f, double beta,
                             double e_reg, double *out, double *out_sum, void *hip_stream) {
    using namespace ami;
    clear_error();
    AmiStatus st = check_common(t, n_e, ext_freqs, n_f, beta, out, out_sum);
    if (st != AMI_OK) return st;
    if (t->n_eps != t->n_g) return fail(AMI_E_ARG, "the momentum path needs one energy per propagator");
    if (t->n_int > kMaxInt) return fail(AMI_E_UNSUPPORTED, "more than 12 summed frequencies on the momentum path");
    if (n_e > 0 && !k) return fail(AMI_E_ARG, "k is NULL");
    if (n_e > 0 && stride_k < 2 * t->n_int) return fail(AMI_E_ARG, "stride_k < 2*n_int");
    if (t->n_ext > 0 && !q) return fail(AMI_E_ARG, "q is NULL");
    FwdParams p;
    std::memset(&p, 0, sizeof(p));
    p.k = k;
    p.stride_k = stride_k;
    for (int x = 0; x < t->n_ext; ++x) {
        p.q[2 * x] = q[2 * x];
        p.q[2 * x + 1] = q[2 * x + 1];
    }
    p.hop_t = hop_t;
    p.mu = mu;
    p.ext_freqs = ext_freqs;
    p.n_f = static_cast<int>(n_f);
    p.beta = beta;
    p.e_reg = e_reg;
    p.n_e = n_e;
    p.out = out;
    return launch_forward(t, true, p, out_sum, static_cast<hipStream_t>(hip_stream));
}

}  // extern "C"
