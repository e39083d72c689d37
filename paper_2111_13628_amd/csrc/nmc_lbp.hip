// Surrogate-Hamiltonian LBP on the CNF factor graph and connected backbone
// growth, for gfx950 (section "Constructing localized surrogate
// Hamiltonians", section "Efficient sampling of localized surrogate
// Hamiltonians via LBP", subsection "4-SAT Problems Near Computational Phase
// Transitions", appendix C; section "Generating backbones of rigid
// variables").
//
// Spins r_i = 2 x_i - 1.  The clause side works in the instance's LBP clause
// order (clauses sorted by their smallest variable, so the clauses of one
// workgroup share variables and their field reads and message writes share
// cache lines): a below is a position in that order, and edge e = 4a + j is
// literal j of the clause there (the clause's spin-table address decodes
// variable and sign; address 2N pads clauses shorter than 4); the variable
// side keeps each variable's incidences in clause-index order.  sigma_e = +1
// for a positive literal.  With the
// field H_i = lambda eps_i s*_i (eps_i = clauses holding i) and the clause
// weight exp(-2 beta) for a violated clause, one message iteration is
//   T_i      = H_i + sum_{b in di} sigma_{ib} u_{b->i}           (per variable)
//   h_{i->a} = sigma_{ia} T_i - u_{a->i}                         (the cavity field)
//   u_{a->i} = -1/2 ln[1 - (1 - e^{-2 beta}) prod_{j in da \ i} (1 - tanh h_{j->a}) / 2]
// The variable kernel (sixteen lanes per variable) writes only T, N doubles
// that stay in L2; the clause kernel (one thread per clause) forms each h
// from T and its own u, so no per-edge h is stored.  Each message is kept
// twice: clause-major (u, the clause kernel's own contiguous reads and
// writes) and variable-major with its sign applied (sigma u at the edge's
// position in the variable's incidence list, written by the clause kernel as
// one scattered 8-byte store), so the variable kernel's sums read contiguous
// memory instead of gathering one cache line per 8-byte message.  The largest
// |du| of an iteration is a workgroup max, then an atomic max over the bit patterns of
// non-negative doubles into one of 64 slots (two sets of slots, by iteration
// parity).  Iterations are queued in batches without host round trips: the
// variable pass of iteration k + 1 first decides on the device whether
// iteration k converged (every wave reads the 64 slots; one thread records
// the decision and clears the other set for the coming clause pass), and
// once stopped the kernels of the rest of the batch return at once, so the
// result is that of checking after every iteration.  A one-thread kernel
// decides on the batch's last iteration.  Everything is fp64 (8 bytes per
// edge and message).
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

// reference spins of one replica, the variable-major position of every edge
// (the variable's incidences in the order of its clause list) and T = H at
// lambda0 (with u = 0 the first clause pass then sees h = sigma H)
__global__ void lbp_setup_kernel(const LbpJob *jobs, double lambda0) {
    const LbpJob &J = jobs[blockIdx.y];
    const KsatDev &I = J.I;
    const LbpWork &W = J.W;
    const uint8_t *xs_row = J.xs_row;
    const int bit = J.bit;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I.n)
        return;
    const int s = ((xs_row[i] >> bit) & 1) ? 1 : -1;
    W.s[i] = (int8_t)s;
    const int q0 = I.var_ptr[i], q1 = I.var_ptr[i + 1];
    W.T[i] = lambda0 * (double)(q1 - q0) * (double)s;
    for (int q = q0; q < q1; ++q) {
        const int a = I.var_cl[q];
        int j = 0;
        for (; j < 3; ++j) {
            const uint32_t ad = I.clause_addr[(size_t)a * 4 + j];
            if (ad == (uint32_t)i || ad == (uint32_t)(i + I.n))
                break;
        }
        W.epos[4 * I.lbp_pos[a] + j] = q;
    }
}

// variable side: T_i; with final != 0 also <r_i> = tanh T_i.  kVarLanes
// lanes share a variable: each takes every kVarLanes-th incidence
// (consecutive lanes read consecutive variable-major messages), the partial
// sums meet by butterfly shuffles inside the lane group.  With gated != 0
// the launch does nothing once the iteration control has stopped; with
// G.judge >= 0 it first decides on the previous iteration (see above) and
// returns without writing T if that iteration ended the step.
constexpr int kVarLanes = 16;
constexpr int kDeltaSlots = kLbpDeltaSlots;
constexpr int kVarRound = 4;

__device__ __forceinline__ int lbp_decide(double d, const LbpJudge &G) {
    return d < G.tol ? 1 : (G.iters >= G.max_iter ? 2 : 0);
}

__global__ void lbp_var_kernel(const LbpJob *jobs, double lambda, int final_pass, int gated, LbpJudge G) {
    const LbpJob &J = jobs[blockIdx.y];
    const KsatDev &I = J.I;
    const LbpWork &W = J.W;
    if (gated && W.ctl[0])
        return;
    if (G.judge >= 0) {
        // the previous iteration's largest |du|: its slots, dealt to the lanes
        unsigned long long mx = 0;
        for (int k = threadIdx.x & 63; k < kDeltaSlots; k += 64) {
            const unsigned long long v = W.scal[G.judge * kDeltaSlots + k];
            mx = v > mx ? v : mx;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(mx, off, 64);
            mx = o > mx ? o : mx;
        }
        const double d = __longlong_as_double((long long)mx);
        const int stop = lbp_decide(d, G);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            W.res[2] = d;
            W.ctl[1] = G.iters;
            W.ctl[0] = stop;
        }
        if (stop)
            return;
    }
    if (G.clear >= 0 && blockIdx.x == 0)
        for (int k = threadIdx.x; k < kDeltaSlots; k += blockDim.x)
            W.scal[G.clear * kDeltaSlots + k] = 0ull;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kVarLanes, l = t % kVarLanes;
    const bool live = i < I.n;
    int q0 = 0, q1 = 0;
    double part = 0.0;
    if (live) {
        q0 = I.var_ptr[i];
        q1 = I.var_ptr[i + 1];
        const double *su = W.uv;
        // four signed messages of the lane per round, in flight together;
        // the lane adds them in incidence order
        for (int q = q0 + l; q < q1; q += kVarRound * kVarLanes) {
            double uv[kVarRound];
#pragma unroll
            for (int k = 0; k < kVarRound; ++k)
                uv[k] = q + k * kVarLanes < q1 ? su[q + k * kVarLanes] : 0.0;
#pragma unroll
            for (int k = 0; k < kVarRound; ++k)
                if (q + k * kVarLanes < q1)
                    part += uv[k];
        }
    }
    for (int off = kVarLanes / 2; off > 0; off >>= 1)
        part += __shfl_xor(part, off, kVarLanes);
    if (!live || l != 0)
        return;
    const double tot = lambda * (double)(q1 - q0) * (double)W.s[i] + part;
    W.T[i] = tot;
    if (final_pass)
        W.mag[i] = tanh(tot);
}

// iteration control at the end of a batch, one thread: the batch's last
// iteration's largest |du| (its set of 64 slots), the iteration count, and
// stop on convergence (ctl[0] = 1) or at max_iter (ctl[0] = 2)
__global__ void lbp_judge_kernel(const LbpJob *jobs, LbpJudge G) {
    const LbpWork &W = jobs[blockIdx.y].W;
    if (W.ctl[0])
        return;
    unsigned long long mx = 0;
    for (int k = 0; k < kDeltaSlots; ++k) {
        const unsigned long long v = W.scal[G.judge * kDeltaSlots + k];
        mx = v > mx ? v : mx;
    }
    const double d = __longlong_as_double((long long)mx);
    W.res[2] = d;
    W.ctl[1] = G.iters;
    W.ctl[0] = lbp_decide(d, G);
}

// clause side: h_{j->a} = sigma_j T_{v_j} - u_{a->j}, then the new u for
// every edge of a and the largest change; with final != 0 the clause moment
// instead (u unchanged)
__global__ void __launch_bounds__(256) lbp_clause_kernel(const LbpJob *jobs, double w, int final_pass, int gated,
                                                         int set) {
    const LbpJob &J = jobs[blockIdx.y];
    const KsatDev &I = J.I;
    const LbpWork &W = J.W;
    if (gated && W.ctl[0])
        return;
    __shared__ double wmax[256 / 64];
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    double dmax = 0.0;
    if (a < I.m) {
        // the clause's four addresses and messages as vector loads, then the
        // four field totals together (a padding slot reads T_0 and drops it)
        const uint4 ad = *reinterpret_cast<const uint4 *>(I.lbp_caddr + (size_t)a * 4);
        double2 *up = reinterpret_cast<double2 *>(W.u + (size_t)a * 4);
        const double2 u01 = up[0], u23 = up[1];
        const uint32_t av[4] = {ad.x, ad.y, ad.z, ad.w};
        const double uo[4] = {u01.x, u01.y, u23.x, u23.y};
        int k = 4;
#pragma unroll
        for (int j = 3; j >= 0; --j)
            if (av[j] >= 2u * (uint32_t)I.n)
                k = j;
        int vj[4];
        double sg[4], tv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool neg = av[j] >= (uint32_t)I.n;
            vj[j] = j < k ? (int)(neg ? av[j] - (uint32_t)I.n : av[j]) : 0;
            sg[j] = neg ? -1.0 : 1.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            tv[j] = W.T[vj[j]];
        double P[4], t[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < k) {
                t[j] = tanh(sg[j] * tv[j] - uo[j]);
                P[j] = (1.0 - t[j]) / 2.0;
            }
        if (!final_pass) {
            double un[4] = {uo[0], uo[1], uo[2], uo[3]};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < k) {
                    double prod = 1.0;
#pragma unroll
                    for (int l = 0; l < 4; ++l)
                        if (l < k && l != j)
                            prod *= P[l];
                    un[j] = -0.5 * log(1.0 - w * prod);
                    const double d = fabs(un[j] - uo[j]);
                    dmax = d > dmax ? d : dmax;
                }
            up[0] = make_double2(un[0], un[1]);
            up[1] = make_double2(un[2], un[3]);
            // the variable-major copies, sign applied (exact)
            const int4 ep = *reinterpret_cast<const int4 *>(W.epos + (size_t)a * 4);
            const int epv[4] = {ep.x, ep.y, ep.z, ep.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < k)
                    W.uv[epv[j]] = sg[j] * un[j];
        } else {
            double sat = 1.0, viol = 1.0, pv = 1.0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < k) {
                    sat *= sg[j] * t[j];
                    viol *= -sg[j] * P[j];
                    pv *= P[j];
                }
            W.corr[a] = (sat - w * viol) / (1.0 - w * pv);
        }
    }
    if (!final_pass) {
        // wave max, workgroup max, one atomic per workgroup into a slot
        for (int off = 32; off > 0; off >>= 1)
            dmax = fmax(dmax, __shfl_xor(dmax, off));
        if ((threadIdx.x & 63) == 0)
            wmax[threadIdx.x >> 6] = dmax;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = wmax[0];
            for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
                m = fmax(m, wmax[k]);
            if (m > 0.0)
                atomic_max_nonneg(&W.scal[set * kDeltaSlots + blockIdx.x % kDeltaSlots], m);
        }
    }
}

// p = (1/N) sum s*_i <r_i> and q1 = (1/N) sum <r_i>^2 in a fixed order
// (one workgroup: strided partial sums, then a tree)
__global__ void __launch_bounds__(1024) lbp_overlap_kernel(const LbpJob *jobs) {
    const KsatDev &I = jobs[blockIdx.y].I;
    const LbpWork &W = jobs[blockIdx.y].W;
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

__global__ void lbp_label_init_kernel(const LbpJob *jobs) {
    const LbpWork &W = jobs[blockIdx.y].W;
    const int n = jobs[blockIdx.y].I.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        W.label[i] = i;
        W.seeded[i] = 0;
        W.size[i] = 0;
    }
}

// every rigid clause lowers its variables' labels to their minimum
__global__ void lbp_hook_kernel(const LbpJob *jobs, double cut) {
    const KsatDev &I = jobs[blockIdx.y].I;
    const LbpWork &W = jobs[blockIdx.y].W;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= I.m || !(fabs(W.corr[a]) >= cut))
        return;
    int vs[4], k = 0, mn = INT32_MAX;
    for (int j = 0; j < 4; ++j) {
        int v;
        double s;
        if (!decode(I.lbp_caddr[(size_t)a * 4 + j], I.n, v, s))
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

__global__ void lbp_jump_kernel(const LbpJob *jobs) {
    const LbpWork &W = jobs[blockIdx.y].W;
    const int n = jobs[blockIdx.y].I.n;
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
__global__ void lbp_seed_kernel(const LbpJob *jobs, double seed_thr) {
    const KsatDev &I = jobs[blockIdx.y].I;
    const LbpWork &W = jobs[blockIdx.y].W;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= I.m || !(fabs(W.corr[a]) >= seed_thr))
        return;
    int v;
    double s;
    if (decode(I.lbp_caddr[(size_t)a * 4], I.n, v, s))
        W.seeded[W.label[v]] = 1;
}

// classes, output labels (-1 outside the backbone) and cluster sizes
__global__ void lbp_classify_kernel(const LbpJob *jobs) {
    const LbpWork &W = jobs[blockIdx.y].W;
    const int n = jobs[blockIdx.y].I.n;
    uint8_t *cls = jobs[blockIdx.y].cls;
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
__global__ void __launch_bounds__(1024) lbp_count_kernel(const LbpJob *jobs, double seed_thr, double cut) {
    const KsatDev &I = jobs[blockIdx.y].I;
    const LbpWork &W = jobs[blockIdx.y].W;
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

// Every launcher covers a batch of jobs (grid y = job); blocks past a job's
// own size return (the clause kernel only after its barriers).
hipError_t lbp_launch_setup(const LbpJob *jobs, const LbpDims &D, double lambda0, hipStream_t s) {
    if (D.max_n > 0)
        hipLaunchKernelGGL(lbp_setup_kernel, dim3(blocks(D.max_n), D.n_jobs), dim3(kLbpThreads), 0, s, jobs, lambda0);
    return hipGetLastError();
}

hipError_t lbp_launch_var(const LbpJob *jobs, const LbpDims &D, double lambda, int final_pass, hipStream_t s) {
    const LbpJudge none{-1, -1, 0, 0, 0.0};
    if (D.max_n > 0)
        hipLaunchKernelGGL(lbp_var_kernel, dim3(blocks(D.max_n * kVarLanes), D.n_jobs), dim3(kLbpThreads), 0, s, jobs,
                           lambda, final_pass, 0, none);
    return hipGetLastError();
}

hipError_t lbp_launch_clause(const LbpJob *jobs, const LbpDims &D, double w, int final_pass, hipStream_t s) {
    if (D.max_m > 0)
        hipLaunchKernelGGL(lbp_clause_kernel, dim3(blocks(D.max_m), D.n_jobs), dim3(kLbpThreads), 0, s, jobs, w,
                           final_pass, 0, 0);
    return hipGetLastError();
}

hipError_t lbp_launch_iterations(const LbpJob *jobs, const LbpDims &D, double lambda, double w, double tol,
                                 int max_iter, int first, int count, hipStream_t s) {
    // iteration k: the variable pass (judging iteration k - 1 within the
    // batch, clearing slot set k & 1), then the clause pass into set k & 1
    for (int k = first; k < first + count; ++k) {
        const LbpJudge G{k > first ? (k - 1) & 1 : -1, k & 1, k, max_iter, tol};
        if (D.max_n > 0)
            hipLaunchKernelGGL(lbp_var_kernel, dim3(blocks(D.max_n * kVarLanes), D.n_jobs), dim3(kLbpThreads), 0, s,
                               jobs, lambda, 0, 1, G);
        if (D.max_m > 0)
            hipLaunchKernelGGL(lbp_clause_kernel, dim3(blocks(D.max_m), D.n_jobs), dim3(kLbpThreads), 0, s, jobs, w, 0,
                               1, k & 1);
    }
    if (count > 0) {
        const int last = first + count - 1;
        hipLaunchKernelGGL(lbp_judge_kernel, dim3(1, D.n_jobs), dim3(1), 0, s, jobs,
                           LbpJudge{last & 1, -1, last + 1, max_iter, tol});
    }
    return hipGetLastError();
}

hipError_t lbp_launch_overlap(const LbpJob *jobs, const LbpDims &D, hipStream_t s) {
    hipLaunchKernelGGL(lbp_overlap_kernel, dim3(1, D.n_jobs), dim3(1024), 0, s, jobs);
    return hipGetLastError();
}

hipError_t lbp_launch_label_init(const LbpJob *jobs, const LbpDims &D, hipStream_t s) {
    if (D.max_n > 0)
        hipLaunchKernelGGL(lbp_label_init_kernel, dim3(blocks(D.max_n), D.n_jobs), dim3(kLbpThreads), 0, s, jobs);
    return hipGetLastError();
}

hipError_t lbp_launch_hook_jump(const LbpJob *jobs, const LbpDims &D, double cut, hipStream_t s) {
    if (D.max_m > 0)
        hipLaunchKernelGGL(lbp_hook_kernel, dim3(blocks(D.max_m), D.n_jobs), dim3(kLbpThreads), 0, s, jobs, cut);
    if (D.max_n > 0)
        hipLaunchKernelGGL(lbp_jump_kernel, dim3(blocks(D.max_n), D.n_jobs), dim3(kLbpThreads), 0, s, jobs);
    return hipGetLastError();
}

hipError_t lbp_launch_finish(const LbpJob *jobs, const LbpDims &D, double seed_thr, double cut, hipStream_t s) {
    if (D.max_m > 0)
        hipLaunchKernelGGL(lbp_seed_kernel, dim3(blocks(D.max_m), D.n_jobs), dim3(kLbpThreads), 0, s, jobs, seed_thr);
    if (D.max_n > 0)
        hipLaunchKernelGGL(lbp_classify_kernel, dim3(blocks(D.max_n), D.n_jobs), dim3(kLbpThreads), 0, s, jobs);
    hipLaunchKernelGGL(lbp_count_kernel, dim3(1, D.n_jobs), dim3(1024), 0, s, jobs, seed_thr, cut);
    return hipGetLastError();
}

}  // namespace nmc
