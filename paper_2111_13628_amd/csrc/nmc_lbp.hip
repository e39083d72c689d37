// Surrogate-Hamiltonian LBP on the CNF factor graph and connected backbone
// growth, for gfx950 (section "Constructing localized surrogate
// Hamiltonians", section "Efficient sampling of localized surrogate
// Hamiltonians via LBP", subsection "4-SAT Problems Near Computational Phase
// Transitions", appendix C; section "Generating backbones of rigid
// variables").
//
// Spins r_i = 2 x_i - 1.  Edge e = 4a + j is literal j of clause a (the
// clause's spin-table address decodes variable and sign; address 2N pads
// clauses shorter than 4).  sigma_e = +1 for a positive literal.  With the
// field H_i = lambda eps_i s*_i (eps_i = clauses holding i) and the clause
// weight exp(-2 beta) for a violated clause, one message iteration is
//   h_{i->a} = sigma_{ia} (H_i + sum_{b in di} sigma_{ib} u_{b->i}) - u_{a->i}
//   u_{a->i} = -1/2 ln[1 - (1 - e^{-2 beta}) prod_{j in da \ i} (1 - tanh h_{j->a}) / 2]
// (the cavity sum as the full sum minus the edge's own term).  One thread
// per variable, then one per clause; the largest |du| of an iteration is an
// atomic max over the bit patterns of non-negative doubles.  Everything is
// fp64: the pass is memory- and latency-bound (8 bytes per edge and message).
//
// Components: labels start as the variable's index; every rigid clause
// (|moment| >= cutoff) lowers its variables' labels to their minimum
// (atomicMin), then labels jump to their label's label, until nothing
// changes.  The fixed point gives every variable of a component the
// component's smallest index.
#include <cmath>

#include "nmc_internal.h"

namespace nmc {

namespace {

constexpr int kLbpThreads = 256;

__device__ __forceinline__ bool decode(uint32_t addr, int n, int &v, double &sg) {
    if (addr >= 2u * (uint32_t)n)
        return false;
    if (addr < (uint32_t)n) {
        v = (int)addr;
        sg = 1.0;
    } else {
        v = (int)addr - n;
        sg = -1.0;
    }
    return true;
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// reference spins of one replica, edge list of every variable (edge | sign
// bit 31, in the order of the variable's clause list), initial h = sigma H
__global__ void lbp_setup_kernel(KsatDev I, const uint8_t *xs_row, int bit, LbpWork W, double lambda0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I.n)
        return;
    const int s = ((xs_row[i] >> bit) & 1) ? 1 : -1;
    W.s[i] = (int8_t)s;
    const int q0 = I.var_ptr[i], q1 = I.var_ptr[i + 1];
    const double H = lambda0 * (double)(q1 - q0) * (double)s;
    for (int q = q0; q < q1; ++q) {
        const int a = I.var_cl[q];
        int j = 0;
        for (; j < 3; ++j) {
            const uint32_t ad = I.clause_addr[(size_t)a * 4 + j];
            if (ad == (uint32_t)i || ad == (uint32_t)(i + I.n))
                break;
        }
        const uint32_t ad = I.clause_addr[(size_t)a * 4 + j];
        const bool neg = ad >= (uint32_t)I.n;
        W.vedge[q] = (4 * a + j) | (neg ? (int)0x80000000 : 0);
        W.h[4 * a + j] = neg ? -H : H;
    }
}

// variable side: h for every edge of i; with final != 0 also <r_i>
__global__ void lbp_var_kernel(KsatDev I, LbpWork W, double lambda, int final_pass) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I.n)
        return;
    const int q0 = I.var_ptr[i], q1 = I.var_ptr[i + 1];
    double tot = lambda * (double)(q1 - q0) * (double)W.s[i];
    for (int q = q0; q < q1; ++q) {
        const int w = W.vedge[q];
        const double u = W.u[w & 0x7FFFFFFF];
        tot += w < 0 ? -u : u;
    }
    for (int q = q0; q < q1; ++q) {
        const int w = W.vedge[q];
        const int e = w & 0x7FFFFFFF;
        W.h[e] = (w < 0 ? -tot : tot) - W.u[e];
    }
    if (final_pass)
        W.mag[i] = tanh(tot);
}

// clause side: new u for every edge of a and the largest change; with
// final != 0 the clause moment instead (u unchanged)
__global__ void lbp_clause_kernel(KsatDev I, LbpWork W, double w, int final_pass) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double dmax = 0.0;
    if (a < I.m) {
        double P[4], t[4], sg[4];
        int k = 0;
        for (int j = 0; j < 4; ++j) {
            int v;
            double s;
            if (!decode(I.clause_addr[(size_t)a * 4 + j], I.n, v, s))
                break;
            t[j] = tanh(W.h[4 * a + j]);
            P[j] = (1.0 - t[j]) / 2.0;
            sg[j] = s;
            k = j + 1;
        }
        if (!final_pass) {
            for (int j = 0; j < k; ++j) {
                double prod = 1.0;
                for (int l = 0; l < k; ++l)
                    if (l != j)
                        prod *= P[l];
                const double un = -0.5 * log(1.0 - w * prod);
                const double d = fabs(un - W.u[4 * a + j]);
                dmax = d > dmax ? d : dmax;
                W.u[4 * a + j] = un;
            }
        } else {
            double sat = 1.0, viol = 1.0, pv = 1.0;
            for (int j = 0; j < k; ++j) {
                sat *= sg[j] * t[j];
                viol *= -sg[j] * P[j];
                pv *= P[j];
            }
            W.corr[a] = (sat - w * viol) / (1.0 - w * pv);
        }
    }
    if (!final_pass) {
        // wave maximum, then one atomic per wave
        for (int off = 32; off > 0; off >>= 1)
            dmax = fmax(dmax, __shfl_xor(dmax, off));
        if ((threadIdx.x & 63) == 0 && dmax > 0.0)
            atomic_max_nonneg(W.scal, dmax);
    }
}

// p = (1/N) sum s*_i <r_i> and q1 = (1/N) sum <r_i>^2 in a fixed order
// (one workgroup: strided partial sums, then a tree)
__global__ void __launch_bounds__(1024) lbp_overlap_kernel(KsatDev I, LbpWork W) {
    __shared__ double sp[1024], sq[1024];
    const int tid = threadIdx.x;
    double p = 0.0, q = 0.0;
    for (int i = tid; i < I.n; i += 1024) {
        const double m = W.mag[i];
        p += (double)W.s[i] * m;
        q += m * m;
    }
    sp[tid] = p;
    sq[tid] = q;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            sp[tid] += sp[tid + w];
            sq[tid] += sq[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        W.res[0] = I.n ? sp[0] / I.n : 1.0;
        W.res[1] = I.n ? sq[0] / I.n : 1.0;
    }
}

__global__ void lbp_label_init_kernel(int n, LbpWork W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        W.label[i] = i;
        W.seeded[i] = 0;
        W.size[i] = 0;
    }
}

// every rigid clause lowers its variables' labels to their minimum
__global__ void lbp_hook_kernel(KsatDev I, LbpWork W, double cut) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= I.m || !(fabs(W.corr[a]) >= cut))
        return;
    int vs[4], k = 0, mn = INT32_MAX;
    for (int j = 0; j < 4; ++j) {
        int v;
        double s;
        if (!decode(I.clause_addr[(size_t)a * 4 + j], I.n, v, s))
            break;
        vs[k++] = v;
        mn = min(mn, W.label[v]);
    }
    bool lowered = false;
    for (int j = 0; j < k; ++j)
        lowered |= atomicMin(&W.label[vs[j]], mn) > mn;
    if (lowered)
        W.flag[0] = 1;
}

__global__ void lbp_jump_kernel(int n, LbpWork W) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int l = W.label[i], ll = W.label[l];
    if (ll < l) {
        W.label[i] = ll;
        W.flag[0] = 1;
    }
}

// seed clauses mark their component
__global__ void lbp_seed_kernel(KsatDev I, LbpWork W, double seed_thr) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= I.m || !(fabs(W.corr[a]) >= seed_thr))
        return;
    int v;
    double s;
    if (decode(I.clause_addr[(size_t)a * 4], I.n, v, s))
        W.seeded[W.label[v]] = 1;
}

// classes, output labels (-1 outside the backbone) and cluster sizes
__global__ void lbp_classify_kernel(int n, LbpWork W, uint8_t *cls) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int l = W.label[i];
    const bool in = W.seeded[l] != 0;
    cls[i] = in ? 1 : 0;
    W.out_label[i] = in ? l : -1;
    if (in)
        atomicAdd(&W.size[l], 1);
}

// backbone size, cluster count, largest cluster, rigid and seed clauses
__global__ void __launch_bounds__(1024) lbp_count_kernel(KsatDev I, LbpWork W, double seed_thr, double cut) {
    __shared__ int s_bb[1024], s_nc[1024], s_mx[1024], s_rg[1024], s_sd[1024];
    const int tid = threadIdx.x;
    int bb = 0, nc = 0, mx = 0, rg = 0, sd = 0;
    for (int i = tid; i < I.n; i += 1024) {
        const int z = W.size[i];
        bb += z;
        nc += z > 0 ? 1 : 0;
        mx = max(mx, z);
    }
    for (int a = tid; a < I.m; a += 1024) {
        const double c = fabs(W.corr[a]);
        rg += c >= cut ? 1 : 0;
        sd += c >= seed_thr ? 1 : 0;
    }
    s_bb[tid] = bb;
    s_nc[tid] = nc;
    s_mx[tid] = mx;
    s_rg[tid] = rg;
    s_sd[tid] = sd;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) {
            s_bb[tid] += s_bb[tid + w];
            s_nc[tid] += s_nc[tid + w];
            s_mx[tid] = max(s_mx[tid], s_mx[tid + w]);
            s_rg[tid] += s_rg[tid + w];
            s_sd[tid] += s_sd[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        W.counts[0] = s_bb[0];
        W.counts[1] = s_nc[0];
        W.counts[2] = s_mx[0];
        W.counts[3] = s_rg[0];
        W.counts[4] = s_sd[0];
    }
}

int blocks(int n) { return (n + kLbpThreads - 1) / kLbpThreads; }

}  // namespace

hipError_t lbp_launch_setup(const KsatDev &I, const uint8_t *xs_row, int bit, const LbpWork &W, double lambda0,
                            hipStream_t s) {
    if (I.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(lbp_setup_kernel, dim3(blocks(I.n)), dim3(kLbpThreads), 0, s, I, xs_row, bit, W, lambda0);
    return hipGetLastError();
}

hipError_t lbp_launch_var(const KsatDev &I, const LbpWork &W, double lambda, int final_pass, hipStream_t s) {
    if (I.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(lbp_var_kernel, dim3(blocks(I.n)), dim3(kLbpThreads), 0, s, I, W, lambda, final_pass);
    return hipGetLastError();
}

hipError_t lbp_launch_clause(const KsatDev &I, const LbpWork &W, double w, int final_pass, hipStream_t s) {
    if (I.m == 0)
        return hipSuccess;
    hipLaunchKernelGGL(lbp_clause_kernel, dim3(blocks(I.m)), dim3(kLbpThreads), 0, s, I, W, w, final_pass);
    return hipGetLastError();
}

hipError_t lbp_launch_overlap(const KsatDev &I, const LbpWork &W, hipStream_t s) {
    hipLaunchKernelGGL(lbp_overlap_kernel, dim3(1), dim3(1024), 0, s, I, W);
    return hipGetLastError();
}

hipError_t lbp_launch_label_init(const KsatDev &I, const LbpWork &W, hipStream_t s) {
    if (I.n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(lbp_label_init_kernel, dim3(blocks(I.n)), dim3(kLbpThreads), 0, s, I.n, W);
    return hipGetLastError();
}

hipError_t lbp_launch_hook_jump(const KsatDev &I, const LbpWork &W, double cut, hipStream_t s) {
    if (I.m > 0)
        hipLaunchKernelGGL(lbp_hook_kernel, dim3(blocks(I.m)), dim3(kLbpThreads), 0, s, I, W, cut);
    if (I.n > 0)
        hipLaunchKernelGGL(lbp_jump_kernel, dim3(blocks(I.n)), dim3(kLbpThreads), 0, s, I.n, W);
    return hipGetLastError();
}

hipError_t lbp_launch_finish(const KsatDev &I, const LbpWork &W, double seed_thr, double cut, uint8_t *cls,
                             hipStream_t s) {
    if (I.m > 0)
        hipLaunchKernelGGL(lbp_seed_kernel, dim3(blocks(I.m)), dim3(kLbpThreads), 0, s, I, W, seed_thr);
    if (I.n > 0)
        hipLaunchKernelGGL(lbp_classify_kernel, dim3(blocks(I.n)), dim3(kLbpThreads), 0, s, I.n, W, cls);
    hipLaunchKernelGGL(lbp_count_kernel, dim3(1), dim3(1024), 0, s, I, W, seed_thr, cut);
    return hipGetLastError();
}

}  // namespace nmc
