// mc_cl.hip -- host runtime and C-ABI of the MI355X Monte Carlo closed-loop
// library (see include/mc_cl.h).  Plans a campaign (per-sample kind, horizon
// and length drawn on the device, NMPC samples grouped by horizon class and
// sorted by work), sizes the persistent NMPC launch from the occupancy the
// kernel reaches, owns the device workspaces and launches every step of the
// path on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "mc_cl.h"
#include "mc_kernels.hpp"
#include "mc_ms.hpp"

using namespace mccl;

namespace {

thread_local std::string g_hip_error;

#define HIPCHK(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) {                                             \
            g_hip_error = std::string(#expr) + ": " + hipGetErrorString(e_); \
            return e_ == hipErrorOutOfMemory ? MC_CL_ENOMEM : MC_CL_EHIP;   \
        }                                                                   \
    } while (0)

// Per-sample plan: kind, horizon and length (device-drawn, as the kernels).
__global__ void plan_kernel(DevParams p, int64_t S, int32_t* kind, int32_t* N, int32_t* L) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    const Setup s = sample_setup(t);
    kind[t] = s.kind;
    N[t] = s.N;
    L[t] = s.L;
}

__global__ void fill_i32(int* a, int n, int v) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = v;
}
__global__ void fill_u64(unsigned long long* a, int n) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = 0ull;
}

// Chunked runs: ctl[0] is the chunk index c; ctl[1 + k] the end of class
// k's groups in chunk c, whose work queue restarts at its first group.
struct ChunkPlan {
    int n_classes;
    int gpc[3], groups[3];
};
__global__ void chunk_begin(int* ctl, int* queue, ChunkPlan cp) {
    const int k = threadIdx.x;
    if (k >= cp.n_classes) return;
    const long long c = ctl[0];
    const long long lo = c * cp.gpc[k], hi = lo + cp.gpc[k];
    queue[k] = (int)(lo < cp.groups[k] ? lo : cp.groups[k]);
    ctl[1 + k] = (int)(hi < cp.groups[k] ? hi : cp.groups[k]);
}
__global__ void chunk_end(int* ctl) {
    if (threadIdx.x == 0) ctl[0] += 1;
}

struct NmpcClass {
    int nmax = 0;
    int64_t count = 0;
    int spw = 64, groups = 0, slots = 0, slots_full = 0;
    int64_t* d_pos = nullptr;
    double* d_tiles = nullptr;
    double* d_xs = nullptr;
    double* d_W = nullptr;
    int64_t tile_stride = 0, xs_stride = 0, w_stride = 0;
    size_t cap_tiles = 0, cap_xs = 0, cap_W = 0;   // allocated elements
};

template <int NMAX, int GMODE, int NX>
hipError_t launch_nmpc(const DevParams& dp, const NmpcWork& wk, const Outs& o, int slots,
                       hipStream_t st) {
    hipLaunchKernelGGL((nmpc_kernel<NMAX, GMODE, NX>), dim3(slots), dim3(64), 0, st, dp, wk, o);
    return hipGetLastError();
}

// Lanes per PI sample (1, 2 or 4; see pi_kernel): the most for which the
// launch keeps at most one wavefront per SIMD (four per compute unit), so
// that wider groups shorten each wavefront's serial chain without queueing
// wavefronts behind one another.  The results do not depend on it.
int pi_lanes(int64_t n, int n_cu) {
    const int64_t simds = 4 * (int64_t)std::max(n_cu, 1);
    for (int k = 4; k > 1; k >>= 1)
        if ((n * k + 63) / 64 <= simds) return k;
    return 1;
}
// The PI forward pass over n samples (a chunk's with ctl, else the first n
// of pos) with k lanes per sample.
hipError_t launch_pi(int k, int64_t n, hipStream_t st, const DevParams& dp, const int64_t* pos,
                     int64_t npi, const Outs& o, double* ck, const int* ctl, int64_t ppc) {
    const dim3 grid((unsigned)((n * k + 63) / 64)), block(64);
    if (k == 4) hipLaunchKernelGGL(pi_kernel<4>, grid, block, 0, st, dp, pos, npi, o, ck, ctl, ppc);
    else if (k == 2) hipLaunchKernelGGL(pi_kernel<2>, grid, block, 0, st, dp, pos, npi, o, ck, ctl, ppc);
    else hipLaunchKernelGGL(pi_kernel<1>, grid, block, 0, st, dp, pos, npi, o, ck, ctl, ppc);
    return hipGetLastError();
}
hipError_t launch_pi_reverse(int k, hipStream_t st, const DevParams& dp, const int64_t* pos,
                             int64_t npi, const double* ck, double* tape, double* ivtape,
                             double* gk) {
    const dim3 grid((unsigned)((npi * k + 63) / 64)), block(64);
    if (k == 4)
        hipLaunchKernelGGL(pi_reverse_kernel<4>, grid, block, 0, st, dp, pos, npi, ck, tape, ivtape, gk);
    else if (k == 2)
        hipLaunchKernelGGL(pi_reverse_kernel<2>, grid, block, 0, st, dp, pos, npi, ck, tape, ivtape, gk);
    else
        hipLaunchKernelGGL(pi_reverse_kernel<1>, grid, block, 0, st, dp, pos, npi, ck, tape, ivtape, gk);
    return hipGetLastError();
}

// Multiple shooting: the horizon class NMAX is the segment width (samples
// per wavefront 64 / NMAX).
template <int G>
hipError_t launch_ms(const DevParams& dp, const NmpcWork& wk, const Outs& o, int slots,
                     hipStream_t st) {
    MsWork mw{wk.pos, wk.n_pos, wk.n_groups, wk.queue, wk.qhi};
    hipLaunchKernelGGL(nmpc_ms_kernel<G>, dim3(slots), dim3(64), 0, st, dp, mw, o);
    return hipGetLastError();
}

template <int G>
int ms_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, nmpc_ms_kernel<G>, 64, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int NMAX, int GMODE, int NX>
int max_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, nmpc_kernel<NMAX, GMODE, NX>, 64, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// Kernel variants: horizon class NMAX x gradient mode x model states; the
// three-state model runs with the adjoint gradient only (validated).
int blocks_per_cu(int nmax, int gmode, int nx, int nlp_form = 0) {
    if (nlp_form == 1)
        return nmax == 16 ? ms_blocks_per_cu<16>() : nmax == 32 ? ms_blocks_per_cu<32>() : ms_blocks_per_cu<64>();
    if (nx == 3) {
        if (nmax == 16) return max_blocks_per_cu<16, 1, 3>();
        if (nmax == 32) return max_blocks_per_cu<32, 1, 3>();
        return max_blocks_per_cu<64, 1, 3>();
    }
    if (gmode == 1) {
        if (nmax == 16) return max_blocks_per_cu<16, 1, 1>();
        if (nmax == 32) return max_blocks_per_cu<32, 1, 1>();
        return max_blocks_per_cu<64, 1, 1>();
    }
    if (nmax == 16) return max_blocks_per_cu<16, 0, 1>();
    if (nmax == 32) return max_blocks_per_cu<32, 0, 1>();
    return max_blocks_per_cu<64, 0, 1>();
}

hipError_t dispatch_nmpc(int nmax, int gmode, int nx, const DevParams& dp, const NmpcWork& wk,
                         const Outs& o, int slots, hipStream_t st) {
    if (dp.nlp_form == 1)
        return nmax == 16 ? launch_ms<16>(dp, wk, o, slots, st)
               : nmax == 32 ? launch_ms<32>(dp, wk, o, slots, st) : launch_ms<64>(dp, wk, o, slots, st);
    if (nx == 3) {
        if (nmax == 16) return launch_nmpc<16, 1, 3>(dp, wk, o, slots, st);
        if (nmax == 32) return launch_nmpc<32, 1, 3>(dp, wk, o, slots, st);
        return launch_nmpc<64, 1, 3>(dp, wk, o, slots, st);
    }
    if (gmode == 1) {
        if (nmax == 16) return launch_nmpc<16, 1, 1>(dp, wk, o, slots, st);
        if (nmax == 32) return launch_nmpc<32, 1, 1>(dp, wk, o, slots, st);
        return launch_nmpc<64, 1, 1>(dp, wk, o, slots, st);
    }
    if (nmax == 16) return launch_nmpc<16, 0, 1>(dp, wk, o, slots, st);
    if (nmax == 32) return launch_nmpc<32, 0, 1>(dp, wk, o, slots, st);
    return launch_nmpc<64, 0, 1>(dp, wk, o, slots, st);
}

bool is_finite(double v) { return std::isfinite(v); }

// Allocation-free runs (mc_cl_run_static): the device memory they use beyond
// the caller's inputs and outputs lives in this file-scope array, one copy
// per device, held until the process ends.  Host code never passes the
// array's name to a kernel: it takes the device address from
// hipGetSymbolAddress once per device (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[MC_CL_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device).
int scratch_ptr(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return MC_CL_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            g_hip_error = "hipGetSymbolAddress returned a null address for the scratch array";
            return MC_CL_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return MC_CL_OK;
}

// Per-sample lists of an allocation-free run, built on the device by one
// block: positions of the NMPC samples of each horizon class (0, 1, 2:
// NMAX 16, 32, 64) and of the PI samples (3), each list in column order,
// stored one after another in `pos`; counts[0..3] the list lengths.
__global__ __launch_bounds__(1024) void bucket_kernel(const int32_t* kind, const int32_t* N,
                                                      int64_t S, int64_t* pos, int* counts) {
    __shared__ int64_t part[4][1024];
    __shared__ int64_t base[4];
    const int t = threadIdx.x;
    const int64_t lo = S * t / 1024, hi = S * (t + 1) / 1024;
    int64_t c[4] = {0, 0, 0, 0};
    auto cls = [&](int64_t s) -> int {
        if (kind[s] == 1) return 3;
        return N[s] <= 16 ? 0 : (N[s] <= 32 ? 1 : 2);
    };
    for (int64_t s = lo; s < hi; ++s) c[cls(s)]++;
    for (int k = 0; k < 4; ++k) part[k][t] = c[k];
    __syncthreads();
    if (t < 4) {
        int64_t run = 0;
        for (int j = 0; j < 1024; ++j) {
            const int64_t v = part[t][j];
            part[t][j] = run;
            run += v;
        }
        base[t] = run;   // class total, turned into list offsets below
    }
    __syncthreads();
    if (t == 0) {
        int64_t off = 0;
        for (int k = 0; k < 4; ++k) {
            counts[k] = (int)base[k];
            const int64_t n = base[k];
            base[k] = off;
            off += n;
        }
    }
    __syncthreads();
    int64_t w[4];
    for (int k = 0; k < 4; ++k) w[k] = base[k] + part[k][t];
    for (int64_t s = lo; s < hi; ++s) pos[w[cls(s)]++] = s;
}

}  // namespace

struct mc_cl_ctx {
    mc_cl_params prm{};
    DevParams dp{};
    int device = 0;
    int n_cu = 0;
    int64_t S = 0;
    int64_t n_pi = 0, n_nmpc = 0;
    std::vector<NmpcClass> classes;
    int* d_queue = nullptr;   // one counter per class
    int* d_ctl = nullptr;     // chunked runs: chunk index, group ends per class
    int n_chunks = 1;
    int64_t pi_per_chunk = 0;
    ChunkPlan cplan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int Lmax = 0;
    int64_t* d_pos_pi = nullptr;
    double* d_phi = nullptr;
    double* d_flops = nullptr;
    int32_t* d_cnt = nullptr;
    uint64_t* d_hash = nullptr;
    double* d_stats = nullptr;
    unsigned long long* d_hist = nullptr;
    long long* d_totals = nullptr;
    // lanes per PI sample chosen by mc_cl_tune (0: pi_lanes' choice)
    int pi_k = 0;
    // PI reverse pass
    int ckC = 0;
    double* d_ck = nullptr;
    double* d_tape = nullptr;
    double* d_ivtape = nullptr;
    double* d_gk = nullptr;
    double* d_gsum = nullptr;
    hipEvent_t ev[6] = {};
    // side streams of the concurrent horizon classes (classes 1 and 2), and
    // the fork/join events that order them against the caller's stream
    hipStream_t side[2] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[2] = {};
    hipStream_t last = nullptr;
    bool ran = false;
    bool grad_ran = false;
    size_t bytes = 0;
    size_t bytes_aligned = 0;   // the same allocations rounded up to 256 bytes each
    std::vector<void*> allocs;

    std::vector<size_t> alloc_bytes;
    // caller-passed workspace (mc_cl_params.workspace): the allocations are
    // carved from it in order, 256-byte aligned, and never freed
    unsigned char* ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;

    template <class T>
    int alloc(T** p, size_t n) {
        *p = nullptr;
        if (n == 0) return MC_CL_OK;
        const size_t b = (n * sizeof(T) + 255) & ~(size_t)255;
        if (ws_base) {
            if (ws_used + b > ws_size) {
                g_hip_error = "caller workspace too small";
                return MC_CL_ENOMEM;
            }
            *p = (T*)(ws_base + ws_used);
            ws_used += b;
            bytes += b;
            bytes_aligned += b;
            return MC_CL_OK;
        }
        void* v = nullptr;
        HIPCHK(hipMalloc(&v, n * sizeof(T)));
        allocs.push_back(v);
        alloc_bytes.push_back(n * sizeof(T));
        bytes += n * sizeof(T);
        bytes_aligned += b;
        *p = (T*)v;
        return MC_CL_OK;
    }
    // Free *p (if the context owns it) and allocate n elements instead (in a
    // caller workspace: a new piece; the old one stays unused).
    template <class T>
    int realloc_dev(T** p, size_t n) {
        if (ws_base) return alloc(p, n);
        for (size_t k = 0; k < allocs.size(); ++k) {
            if (allocs[k] == (void*)*p && *p) {
                HIPCHK(hipFree(allocs[k]));
                bytes -= alloc_bytes[k];
                allocs.erase(allocs.begin() + k);
                alloc_bytes.erase(alloc_bytes.begin() + k);
                break;
            }
        }
        return alloc(p, n);
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
    ~mc_cl_ctx() {
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        drop_graph();
        for (void* v : allocs) (void)hipFree(v);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& sd : side)
            if (sd) (void)hipStreamDestroy(sd);
        if (fork) (void)hipEventDestroy(fork);
        for (auto& e : join)
            if (e) (void)hipEventDestroy(e);
    }
    // The side streams and events, created on first use (default priority,
    // not blocking on the null stream).
    int ensure_side() {
        if (fork) return MC_CL_OK;
        for (auto& sd : side) HIPCHK(hipStreamCreateWithFlags(&sd, hipStreamNonBlocking));
        for (auto& e : join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        return MC_CL_OK;
    }
};

// Lanes per PI sample for a launch over n samples: the tuned choice, else
// pi_lanes' rule.
static int pi_k_of(const mc_cl_ctx* c, int64_t n) { return c->pi_k > 0 ? c->pi_k : pi_lanes(n, c->n_cu); }

static int validate(const mc_cl_params* p) {
    if (!p) return MC_CL_EINVAL;
    if (p->struct_size != sizeof(mc_cl_params) || p->abi_version != MC_CL_ABI_VERSION)
        return MC_CL_EINVAL;
    const double fin[] = {p->V, p->k0, p->EaR, p->beta, p->cAin, p->cBin, p->cTin, p->sigma[0],
                          p->sigma[1], p->sigma[2], p->Rmeas, p->Ts, p->Qz, p->umin, p->umax,
                          p->sqp_eps, p->ls_c1, p->ls_beta, p->kP, p->kI, p->kaw, p->pi_umin,
                          p->pi_umax, p->P0, p->x0_rel_std, p->sp_step_rel, p->kin_lognorm_sigma,
                          p->noise_scale};
    for (double v : fin)
        if (!is_finite(v)) return MC_CL_EINVAL;
    if (!(p->V > 0) || !(p->Ts > 0) || !(p->beta != 0) || !(p->k0 >= 0) || !(p->EaR > 0))
        return MC_CL_EINVAL;
    if (p->Ns < 1 || p->Nc < 1 || p->L < 0 || p->n_samples < 1) return MC_CL_EINVAL;
    if (p->N < 1 || p->N > MC_CL_NMAX || p->umin > p->umax || p->pi_umin > p->pi_umax)
        return MC_CL_EINVAL;
    if (p->Rmeas < 0 || p->P0 <= 0 || p->sigma[0] < 0 || p->sigma[1] < 0 || p->sigma[2] < 0)
        return MC_CL_EINVAL;
    if (p->n_sp < 1 || p->n_sp > MC_CL_SPMAX || p->sp_i[0] != 0) return MC_CL_EINVAL;
    for (int j = 0; j < p->n_sp; ++j) {
        if (!is_finite(p->sp_z[j]) || p->sp_z[j] <= p->cTin) return MC_CL_EINVAL;
        if (j > 0 && p->sp_i[j] <= p->sp_i[j - 1]) return MC_CL_EINVAL;
    }
    if (p->sp_period < 0) return MC_CL_EINVAL;
    if (p->sp_step_rel != 0.0 && (p->sp_step_lo < 0 || p->sp_step_hi < p->sp_step_lo))
        return MC_CL_EINVAL;
    if (p->n_horizon_choices < 0 || p->n_horizon_choices > 4) return MC_CL_EINVAL;
    for (int j = 0; j < p->n_horizon_choices; ++j)
        if (p->horizon_choices[j] < 1 || p->horizon_choices[j] > MC_CL_NMAX) return MC_CL_EINVAL;
    if (p->L_lo < p->L_hi && p->L_lo < 0) return MC_CL_EINVAL;
    if (p->sqp_max_iter < 0 || p->ls_max_bt < 0 || p->ipm_max_iter < 1) return MC_CL_EINVAL;
    if (p->grad_mode != 0 && p->grad_mode != 1) return MC_CL_EINVAL;
    if (p->x0_mode != 0 && p->x0_mode != 1) return MC_CL_EINVAL;
    if (p->default_kind != 0 && p->default_kind != 1) return MC_CL_EINVAL;
    if (!(p->ls_beta > 0 && p->ls_beta < 1) || !(p->ls_c1 > 0 && p->ls_c1 < 1)) return MC_CL_EINVAL;
    if (p->kP == 0.0 || p->kI == 0.0) return MC_CL_EINVAL;
    if (p->ckpt_interval < 0 || p->samples_per_wave < 0 || p->samples_per_wave > 64)
        return MC_CL_EINVAL;
    if (p->qp_solver < 0 || p->qp_solver > 2) return MC_CL_EINVAL;
    if (p->chunk_samples < 0 || p->cu_limit < 0) return MC_CL_EINVAL;
    if (p->model_nx != 1 && p->model_nx != 3) return MC_CL_EINVAL;
    if (p->model_nx == 3 && p->grad_mode != 1) return MC_CL_EUNSUPPORTED;
    if (p->nlp_form != 0 && p->nlp_form != 1) return MC_CL_EINVAL;
    if (p->nlp_form == 1 && !(p->umin < p->umax)) return MC_CL_EINVAL;
    if (p->nlp_form == 1 && p->model_nx != 1) return MC_CL_EUNSUPPORTED;
    if (p->workspace && (p->workspace_size == 0 || ((uintptr_t)p->workspace & 255u) != 0))
        return MC_CL_EINVAL;
    if (p->class_streams != 0 && p->class_streams != 1) return MC_CL_EINVAL;
    if (!p->sample_ids &&
        (p->sample_id_offset < 0 || p->sample_id_offset + p->n_samples > (int64_t)UINT32_MAX))
        return MC_CL_EINVAL;
    for (int64_t s = 0; s < p->n_samples; ++s) {
        if (p->sample_ids && (p->sample_ids[s] < 0 || p->sample_ids[s] >= (int64_t)UINT32_MAX))
            return MC_CL_EINVAL;
        if (p->kind && p->kind[s] > 1) return MC_CL_EINVAL;
        if (p->horizon && (p->horizon[s] < 1 || p->horizon[s] > MC_CL_NMAX)) return MC_CL_EINVAL;
        if (p->lengths && (p->lengths[s] < 0 || p->lengths[s] > (1 << 24))) return MC_CL_EINVAL;
    }
    return MC_CL_OK;
}

// Launch shape of an NMPC class for `spw` samples per wavefront; grows the
// class's wave-slot workspaces when the shape needs more of them.
static int plan_class(mc_cl_ctx* c, NmpcClass& nc, int spw) {
    const bool ms = c->prm.nlp_form == 1;
    // multiple shooting: the queue hands out single samples, each taken by
    // an NMAX-lane segment (a stage per lane), 64 / NMAX segments per wavefront
    if (ms) spw = 1;
    nc.spw = spw;
    nc.groups = (int)((nc.count + spw - 1) / spw);
    const int per_wave = ms ? 64 / nc.nmax : 1;
    nc.slots = std::min((nc.groups + per_wave - 1) / per_wave, nc.slots_full);
    // multiple shooting keeps every stage quantity in registers
    nc.tile_stride = ms ? 0 : (int64_t)V_COUNT * nc.nmax * 64;
    nc.xs_stride = ms ? 0 : (int64_t)(c->prm.model_nx == 3 ? rec_width<3>() : rec_width<1>()) * nc.nmax * 64;
    nc.w_stride = ms ? 0 : (int64_t)spw * nc.nmax * nc.nmax;
    const size_t nt = (size_t)nc.slots * nc.tile_stride;
    const size_t nx = (size_t)nc.slots * nc.xs_stride;
    const size_t nw = (size_t)nc.slots * nc.w_stride;
    int rc;
    if (nt > nc.cap_tiles) {
        if ((rc = c->realloc_dev(&nc.d_tiles, nt))) return rc;
        nc.cap_tiles = nt;
    }
    if (nx > nc.cap_xs) {
        if ((rc = c->realloc_dev(&nc.d_xs, nx))) return rc;
        nc.cap_xs = nx;
    }
    if (nw > nc.cap_W) {
        if ((rc = c->realloc_dev(&nc.d_W, nw))) return rc;
        nc.cap_W = nw;
        HIPCHK(hipMemset(nc.d_W, 0, nw * 8));
    }
    return MC_CL_OK;
}

// PI reverse-pass buffers for checkpoints every C intervals: the plant
// states at the segment starts, and one segment's sub-step and interval
// tapes.
static int size_ckpt(mc_cl_ctx* c, int C) {
    const int64_t nseg = std::max<int64_t>((c->Lmax + C - 1) / C, 1);
    int rc;
    if ((rc = c->realloc_dev(&c->d_ck, (size_t)nseg * 4 * c->n_pi)) ||
        (rc = c->realloc_dev(&c->d_tape, (size_t)C * c->prm.Ns * 6 * c->n_pi)) ||
        (rc = c->realloc_dev(&c->d_ivtape, (size_t)C * 5 * c->n_pi)))
        return rc;
    c->ckC = C;
    c->dp.ckpt_C = C;
    return MC_CL_OK;
}

// Work of each chunk: a contiguous range of every class's groups and of
// the PI samples.
static void set_chunk_plan(mc_cl_ctx* c) {
    const int nch = std::max(c->n_chunks, 1);
    c->cplan.n_classes = (int)c->classes.size();
    for (size_t k = 0; k < c->classes.size(); ++k) {
        c->cplan.groups[k] = c->classes[k].groups;
        c->cplan.gpc[k] = (c->classes[k].groups + nch - 1) / nch;
    }
    c->pi_per_chunk = (c->n_pi + nch - 1) / nch;
}

// One campaign step on `st`: every NMPC class's persistent launch, then the
// PI launch.  With chunk set the step covers chunk ctl[0] only and ends by
// advancing it (the sequence captured in the run graph).  `ev_mid` (or
// null) is recorded between the NMPC and PI launches.
static int launch_step(mc_cl_ctx* c, hipStream_t st, const Outs& out, bool chunk,
                       hipEvent_t ev_mid) {
    if (chunk) {
        hipLaunchKernelGGL(chunk_begin, dim3(1), dim3(64), 0, st, c->d_ctl, c->d_queue, c->cplan);
        HIPCHK(hipGetLastError());
    } else {
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, c->d_queue, 4, 0);
        HIPCHK(hipGetLastError());
    }
    // With class_streams the horizon classes run concurrently (unchunked
    // runs on the whole device): the waves of one class's launch take the
    // SIMDs that another's tail leaves idle, as one persistent launch over
    // all classes would.  Their queues, workspaces and output positions are
    // disjoint.  Otherwise one after another on `st`.
    const bool conc = !chunk && c->classes.size() > 1 && c->prm.cu_limit == 0 &&
                      c->prm.class_streams == 1 && c->fork;
    if (conc) {
        HIPCHK(hipEventRecord(c->fork, st));
        for (size_t k = 1; k < c->classes.size(); ++k)
            HIPCHK(hipStreamWaitEvent(c->side[k - 1], c->fork, 0));
    }
    for (size_t k = 0; k < c->classes.size(); ++k) {
        const NmpcClass& nc = c->classes[k];
        NmpcWork wk{nc.d_pos, nc.count, nc.spw, nc.groups, c->d_queue + k,
                    chunk ? c->d_ctl + 1 + k : nullptr, nc.d_tiles, nc.d_xs, nc.d_W,
                    nc.tile_stride, nc.xs_stride, nc.w_stride};
        HIPCHK(dispatch_nmpc(nc.nmax, c->prm.grad_mode, c->prm.model_nx, c->dp, wk, out, nc.slots,
                             conc && k > 0 ? c->side[k - 1] : st));
    }
    if (conc) {
        for (size_t k = 1; k < c->classes.size(); ++k) {
            HIPCHK(hipEventRecord(c->join[k - 1], c->side[k - 1]));
            HIPCHK(hipStreamWaitEvent(st, c->join[k - 1], 0));
        }
    }
    if (ev_mid) HIPCHK(hipEventRecord(ev_mid, st));
    if (c->n_pi) {
        const int64_t n = chunk ? c->pi_per_chunk : c->n_pi;
        HIPCHK(launch_pi(pi_k_of(c, n), n, st, c->dp, c->d_pos_pi, c->n_pi, out, c->d_ck,
                         chunk ? c->d_ctl : nullptr, c->pi_per_chunk));
    }
    if (chunk) {
        hipLaunchKernelGGL(chunk_end, dim3(1), dim3(64), 0, st, c->d_ctl);
        HIPCHK(hipGetLastError());
    }
    return MC_CL_OK;
}

// Capture one chunk step into a graph and instantiate it.
static int capture_step(mc_cl_ctx* c, const Outs& out) {
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int rc = MC_CL_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        g_hip_error = "hipStreamBeginCapture failed";
        rc = MC_CL_EHIP;
    } else {
        rc = launch_step(c, cs, out, true, nullptr);
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc == MC_CL_OK && e != hipSuccess) {
            g_hip_error = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
            rc = MC_CL_EHIP;
        }
    }
    if (rc == MC_CL_OK) {
        const hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            g_hip_error = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
            rc = MC_CL_EHIP;
        }
    }
    if (rc == MC_CL_OK) c->graph = g;
    else if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    return rc;
}

static DevParams to_dev(const mc_cl_params& p) {
    DevParams d{};
    d.V = p.V; d.k0 = p.k0; d.EaR = p.EaR; d.beta = p.beta;
    d.cAin = p.cAin; d.cBin = p.cBin; d.cTin = p.cTin;
    for (int a = 0; a < 3; ++a) d.sig[a] = p.sigma[a];
    d.Rmeas = p.Rmeas; d.Ts = p.Ts; d.Ns = p.Ns; d.L = p.L;
    d.n_sp = p.n_sp; d.sp_period = p.sp_period;
    for (int j = 0; j < kSpMax; ++j) { d.sp_i[j] = p.sp_i[j]; d.sp_z[j] = p.sp_z[j]; }
    d.sp_step_rel = p.sp_step_rel; d.sp_step_lo = p.sp_step_lo; d.sp_step_hi = p.sp_step_hi;
    d.N = p.N; d.Nc = p.Nc; d.Qz = p.Qz; d.umin = p.umin; d.umax = p.umax;
    d.sqp_eps = p.sqp_eps; d.ls_c1 = p.ls_c1; d.ls_beta = p.ls_beta;
    d.sqp_max_iter = p.sqp_max_iter; d.ls_max_bt = p.ls_max_bt; d.grad_mode = p.grad_mode;
    d.ipm_max_iter = p.ipm_max_iter;
    d.kP = p.kP; d.kI = p.kI; d.kaw = p.kaw; d.pi_umin = p.pi_umin; d.pi_umax = p.pi_umax;
    d.P0 = p.P0; d.x0_rel_std = p.x0_rel_std; d.x0_mode = p.x0_mode;
    d.kind_split = p.kind_split; d.default_kind = p.default_kind;
    d.run_ekf_for_pi = p.run_ekf_for_pi;
    d.seed = p.seed; d.noise_mod = p.noise_mod; d.n_samples = p.n_samples;
    d.id_offset = p.sample_id_offset;
    d.n_hc = p.n_horizon_choices;
    for (int j = 0; j < 4; ++j) d.hc[j] = p.horizon_choices[j];
    d.L_lo = p.L_lo; d.L_hi = p.L_hi; d.kin_sigma = p.kin_lognorm_sigma;
    d.hess_warm = p.hess_warm; d.want_grad = p.want_grad; d.noise_scale = p.noise_scale;
    d.ckpt_C = 0;
    d.qp_solver = p.qp_solver;
    d.L_cap = INT32_MAX;
    d.model_nx = p.model_nx;
    d.ids = nullptr;       // device copies of the per-sample arrays: set at create
    d.kind_ov = nullptr;
    d.N_ov = nullptr;
    d.L_ov = nullptr;
    d.nlp_form = p.nlp_form;
    return d;
}

static int nmax_class(int N) { return N <= 16 ? 16 : (N <= 32 ? 32 : 64); }

// Samples per wavefront.  Per SQP iteration a wavefront spends a time in the
// one-sample-per-lane phases that does not depend on how many of its lanes
// carry samples (their serial RK4 chains are latency bound), plus one
// cooperative visit (BFGS update and QP) per sample.  With
// rho = T_lane / T_visit (measured on MI355X with the inverse-form QP: about
// 85 at N = 60, scaling like 60 / N since the lane phases grow with N and
// the visit with N^2), the campaign rate is proportional to
// resident_waves(spw) * spw / (rho + spw).  Pick the best of 1..64.
static int choose_spw(int64_t count, int N, int slots_full) {
    const double rho = 85.0 * 60.0 / (double)std::max(N, 1);
    int best = 64;
    double best_rate = -1.0;
    for (int spw = 64; spw >= 1; spw >>= 1) {
        const int64_t groups = (count + spw - 1) / spw;
        const double resident = (double)std::min<int64_t>(groups, slots_full);
        const double rate = resident * spw / (rho + spw);
        if (rate > best_rate * 1.02) {
            best_rate = rate;
            best = spw;
        }
    }
    return best;
}

// Samples per wavefront evened out over the wave slots: `spw` is a cap, and
// the groups are made as small as the same number of rounds (groups per
// resident wavefront, rounded up) allows.  A wavefront's lane phases take
// the same time however many of its lanes carry samples, and its visits are
// serial over its samples, so fewer samples per wavefront only shortens
// each wavefront (c1: 938 groups of 32 on 1,024 slots become 1,000 groups
// of 30; c4: 7,813 groups of 64 in 8 rounds become 8,065 of 62).  With
// several rounds the groups are shrunk by at most an eighth: much smaller
// groups add lock-step rounds (each group runs an interval's SQP until its
// slowest sample is done), which cost more than the filled last round saves
// (c3's N = 50 class, 32 to 17 per group: 2 % slower).
static int balanced_spw(int64_t count, int spw, int slots_full) {
    const int64_t groups = (count + spw - 1) / spw;
    const int64_t cap = (int64_t)std::max(slots_full, 1);
    const int64_t rounds = (groups + cap - 1) / cap;
    const int64_t b = std::max<int64_t>(1, (count + rounds * cap - 1) / (rounds * cap));
    if (rounds > 1 && 8 * b < 7 * (int64_t)spw) return spw;
    return (int)std::min<int64_t>(spw, b);
}

extern "C" {

uint32_t mc_cl_abi_version(void) { return MC_CL_ABI_VERSION; }

const char* mc_cl_strerror(int status) {
    switch (status) {
        case MC_CL_OK: return "ok";
        case MC_CL_EINVAL: return "invalid argument or parameter out of domain";
        case MC_CL_EHIP: return g_hip_error.empty() ? "HIP runtime error" : g_hip_error.c_str();
        case MC_CL_ENOMEM: return "device allocation failed";
        case MC_CL_ESTATE: return "call out of order for this context";
        case MC_CL_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

int mc_cl_create(const mc_cl_params* p, mc_cl_ctx** out) {
    if (!out) return MC_CL_EINVAL;
    int rc = validate(p);
    if (rc != MC_CL_OK) return rc;
    mc_cl_ctx* c = new (std::nothrow) mc_cl_ctx();
    if (!c) return MC_CL_ENOMEM;
    auto fail = [&](int code) {
        delete c;
        return code;
    };
    c->prm = *p;
    c->dp = to_dev(*p);
    c->S = p->n_samples;
    if (p->workspace) {
        c->ws_base = (unsigned char*)p->workspace;
        c->ws_size = p->workspace_size;
    }
    c->prm.workspace = nullptr;   // the context keeps its own record of it
    if (hipGetDevice(&c->device) != hipSuccess) return fail(MC_CL_EHIP);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return fail(MC_CL_EHIP);
    c->n_cu = prop.multiProcessorCount;
    if (p->cu_limit > 0 && p->cu_limit < c->n_cu) c->n_cu = p->cu_limit;
    const int64_t S = c->S;
    // the caller's per-sample arrays, copied to the device (the context's
    // parameter copy must not keep the caller's host pointers)
    c->prm.sample_ids = nullptr;
    c->prm.kind = nullptr;
    c->prm.horizon = nullptr;
    c->prm.lengths = nullptr;
    if (p->sample_ids) {
        int64_t* d = nullptr;
        if ((rc = c->alloc(&d, S))) return fail(rc);
        if (hipMemcpy(d, p->sample_ids, S * 8, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MC_CL_EHIP);
        c->dp.ids = d;
    }
    if (p->kind) {
        uint8_t* d = nullptr;
        if ((rc = c->alloc(&d, S))) return fail(rc);
        if (hipMemcpy(d, p->kind, S, hipMemcpyHostToDevice) != hipSuccess) return fail(MC_CL_EHIP);
        c->dp.kind_ov = d;
    }
    if (p->horizon) {
        int32_t* d = nullptr;
        if ((rc = c->alloc(&d, S))) return fail(rc);
        if (hipMemcpy(d, p->horizon, S * 4, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MC_CL_EHIP);
        c->dp.N_ov = d;
    }
    if (p->lengths) {
        int32_t* d = nullptr;
        if ((rc = c->alloc(&d, S))) return fail(rc);
        if (hipMemcpy(d, p->lengths, S * 4, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MC_CL_EHIP);
        c->dp.L_ov = d;
    }

    // plan: per-sample kind / N / L on the device
    int32_t *d_kind, *d_N, *d_L;
    if ((rc = c->alloc(&d_kind, S)) || (rc = c->alloc(&d_N, S)) || (rc = c->alloc(&d_L, S)))
        return fail(rc);
    hipLaunchKernelGGL(plan_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, 0, c->dp, S,
                       d_kind, d_N, d_L);
    std::vector<int32_t> kind(S), Nv(S), Lv(S);
    if (hipMemcpy(kind.data(), d_kind, S * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(Nv.data(), d_N, S * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(Lv.data(), d_L, S * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MC_CL_EHIP);
    std::vector<int64_t> pi_pos;
    std::vector<std::vector<int64_t>> cls_pos(3);
    int Lmax = 0;
    for (int64_t s = 0; s < S; ++s) {
        Lmax = std::max(Lmax, Lv[s]);
        if (kind[s] == 1) pi_pos.push_back(s);
        else cls_pos[nmax_class(Nv[s]) == 16 ? 0 : (nmax_class(Nv[s]) == 32 ? 1 : 2)].push_back(s);
    }
    c->n_pi = (int64_t)pi_pos.size();
    if (c->n_pi) {
        if ((rc = c->alloc(&c->d_pos_pi, c->n_pi))) return fail(rc);
        if (hipMemcpy(c->d_pos_pi, pi_pos.data(), c->n_pi * 8, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MC_CL_EHIP);
    }
    // NMPC classes: sorted by (N, L) descending so a wavefront's samples
    // carry similar work
    const int gmode = p->grad_mode;
    const int nmaxs[3] = {16, 32, 64};
    for (int k = 0; k < 3; ++k) {
        auto& v = cls_pos[k];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [&](int64_t a, int64_t b) {
            if (Nv[a] != Nv[b]) return Nv[a] > Nv[b];
            return Lv[a] > Lv[b];
        });
        NmpcClass nc;
        nc.nmax = nmaxs[k];
        nc.count = (int64_t)v.size();
        c->n_nmpc += nc.count;
        const int bpc = blocks_per_cu(nc.nmax, gmode, p->model_nx, p->nlp_form);
        nc.slots_full = bpc * c->n_cu;
        int nmax_in_class = 1;
        for (int64_t q : v) nmax_in_class = std::max(nmax_in_class, Nv[q]);
        const int spw = p->samples_per_wave > 0 ? p->samples_per_wave
                                                : balanced_spw(nc.count,
                                                               choose_spw(nc.count, nmax_in_class,
                                                                          nc.slots_full),
                                                               nc.slots_full);
        if ((rc = c->alloc(&nc.d_pos, nc.count)) || (rc = plan_class(c, nc, spw))) return fail(rc);
        if (hipMemcpy(nc.d_pos, v.data(), nc.count * 8, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MC_CL_EHIP);
        c->classes.push_back(nc);
    }
    c->Lmax = Lmax;
    if ((rc = c->alloc(&c->d_queue, 4)) || (rc = c->alloc(&c->d_ctl, 4)) ||
        (rc = c->alloc(&c->d_phi, S)) ||
        (rc = c->alloc(&c->d_flops, S)) || (rc = c->alloc(&c->d_cnt, (size_t)C_NCNT * S)) ||
        (rc = c->alloc(&c->d_hash, S)) || (rc = c->alloc(&c->d_stats, 8)) ||
        (rc = c->alloc(&c->d_hist, 2 * MC_CL_NHIST)) || (rc = c->alloc(&c->d_totals, MC_CL_NCNT)))
        return fail(rc);
    if (p->want_grad && c->n_pi) {
        if ((rc = size_ckpt(c, p->ckpt_interval > 0 ? p->ckpt_interval : 50)) ||
            (rc = c->alloc(&c->d_gk, (size_t)2 * c->n_pi)) || (rc = c->alloc(&c->d_gsum, 2)))
            return fail(rc);
    }
    if (p->chunk_samples > 0)
        c->n_chunks = (int)std::max<int64_t>(1, (S + p->chunk_samples - 1) / p->chunk_samples);
    set_chunk_plan(c);
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(MC_CL_EHIP);
    *out = c;
    return MC_CL_OK;
}

int mc_cl_run(mc_cl_ctx* c, void* hip_stream, const mc_cl_outputs* o) {
    if (!c) return MC_CL_EINVAL;
    const bool traj = o && (o->traj_z || o->traj_u || o->traj_xhat);
    const bool chunked = c->n_chunks > 1;
    if (traj && chunked) return MC_CL_EUNSUPPORTED;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    Outs out{c->d_phi, c->d_flops, c->d_cnt, c->d_hash,
             o ? o->traj_z : nullptr, o ? o->traj_u : nullptr, o ? o->traj_xhat : nullptr, c->S};
    hipLaunchKernelGGL(fill_u64, dim3((2 * MC_CL_NHIST + MC_CL_NCNT + 255) / 256), dim3(256), 0,
                       st, c->d_hist, 2 * MC_CL_NHIST);
    hipLaunchKernelGGL(fill_u64, dim3(1), dim3(64), 0, st, (unsigned long long*)c->d_totals,
                       MC_CL_NCNT);
    HIPCHK(hipGetLastError());
    if (chunked) {
        // the captured chunk step, replayed once per chunk; it starts from
        // chunk 0 and advances the device-side chunk index itself
        if (!c->gexec) {
            const int rc = capture_step(c, out);
            if (rc != MC_CL_OK) return rc;
        }
        hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, c->d_ctl, 4, 0);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(c->ev[0], st));
        for (int k = 0; k < c->n_chunks; ++k) HIPCHK(hipGraphLaunch(c->gexec, st));
        HIPCHK(hipEventRecord(c->ev[1], st));
    } else {
        if (c->classes.size() > 1 && c->prm.cu_limit == 0 && c->prm.class_streams == 1) {
            const int rc = c->ensure_side();
            if (rc != MC_CL_OK) return rc;
        }
        HIPCHK(hipEventRecord(c->ev[0], st));
        const int rc = launch_step(c, st, out, false, c->ev[1]);
        if (rc != MC_CL_OK) return rc;
    }
    HIPCHK(hipEventRecord(c->ev[2], st));
    hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(1024), 0, st, c->d_phi, c->d_cnt, c->S,
                       c->d_flops, c->d_stats, c->d_hist, c->d_totals);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev[3], st));
    if (o) {
        if (o->phi) HIPCHK(hipMemcpyAsync(o->phi, c->d_phi, c->S * 8, hipMemcpyDeviceToDevice, st));
        if (o->counters)
            HIPCHK(hipMemcpyAsync(o->counters, c->d_cnt, (size_t)C_NCNT * c->S * 4,
                                  hipMemcpyDeviceToDevice, st));
        if (o->ashash)
            HIPCHK(hipMemcpyAsync(o->ashash, c->d_hash, c->S * 8, hipMemcpyDeviceToDevice, st));
    }
    c->last = st;
    c->ran = true;
    return MC_CL_OK;
}

int mc_cl_costs(mc_cl_ctx* c, double* phi_host, mc_cl_stats* sto) {
    if (!c) return MC_CL_EINVAL;
    if (!c->ran) return MC_CL_ESTATE;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->last));
    if (phi_host) HIPCHK(hipMemcpy(phi_host, c->d_phi, c->S * 8, hipMemcpyDeviceToHost));
    if (sto) {
        double s8[8];
        unsigned long long hist[2 * MC_CL_NHIST];
        long long tot[MC_CL_NCNT];
        HIPCHK(hipMemcpy(s8, c->d_stats, sizeof(s8), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hist, c->d_hist, sizeof(hist), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(tot, c->d_totals, sizeof(tot), hipMemcpyDeviceToHost));
        std::memset(sto, 0, sizeof(*sto));
        for (int k = 0; k < 2; ++k) {
            sto->count[k] = (int64_t)s8[k * 3 + 0];
            sto->mean[k] = s8[k * 3 + 1];
            sto->var[k] = s8[k * 3 + 2];
            for (int b = 0; b < MC_CL_NHIST; ++b) sto->hist[k][b] = (int64_t)hist[k * MC_CL_NHIST + b];
        }
        for (int r = 0; r < MC_CL_NCNT; ++r) sto->totals[r] = tot[r];
        sto->flops_algorithmic = s8[6] + s8[7];
        sto->flops_by_kind[0] = s8[6];
        sto->flops_by_kind[1] = s8[7];
        sto->workspace_bytes = c->bytes;
    }
    return MC_CL_OK;
}

int mc_cl_grad(mc_cl_ctx* c, void* hip_stream, double g[2], double* per_sample) {
    if (!c || !g) return MC_CL_EINVAL;
    if (!c->ran || !c->prm.want_grad || c->n_pi == 0 || !c->d_ck) return MC_CL_ESTATE;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    HIPCHK(hipEventRecord(c->ev[4], st));
    HIPCHK(launch_pi_reverse(pi_k_of(c, c->n_pi), st, c->dp, c->d_pos_pi, c->n_pi, c->d_ck,
                             c->d_tape, c->d_ivtape, c->d_gk));
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(1), dim3(1024), 0, st, c->d_gk, c->n_pi, c->d_gsum);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(c->ev[5], st));
    c->grad_ran = true;
    double gs[2];
    HIPCHK(hipMemcpyAsync(gs, c->d_gsum, sizeof(gs), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // theta = (Kc, tau_i), kP = Kc, kI = Kc / tau_i
    const double Kc = c->prm.kP, taui = c->prm.kP / c->prm.kI;
    const double dkP = gs[0] / (double)c->n_pi, dkI = gs[1] / (double)c->n_pi;
    g[0] = dkP + dkI / taui;
    g[1] = dkI * (-Kc / (taui * taui));
    if (per_sample) {
        // per-sample (Kc, tau_i) derivatives at the sample columns; zero for NMPC
        std::vector<double> gk(2 * c->n_pi), ps(2 * c->S, 0.0);
        std::vector<int64_t> pos(c->n_pi);
        HIPCHK(hipMemcpy(gk.data(), c->d_gk, gk.size() * 8, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(pos.data(), c->d_pos_pi, pos.size() * 8, hipMemcpyDeviceToHost));
        for (int64_t t = 0; t < c->n_pi; ++t) {
            ps[pos[t]] = gk[t] + gk[c->n_pi + t] / taui;
            ps[c->S + pos[t]] = gk[c->n_pi + t] * (-Kc / (taui * taui));
        }
        HIPCHK(hipMemcpy(per_sample, ps.data(), ps.size() * 8, hipMemcpyHostToDevice));
    }
    return MC_CL_OK;
}

void mc_cl_destroy(mc_cl_ctx* c) { delete c; }

int mc_cl_kernel_ms(mc_cl_ctx* c, float ms[4]) {
    if (!c || !ms || !c->ran) return MC_CL_ESTATE;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipEventSynchronize(c->ev[3]));
    HIPCHK(hipEventElapsedTime(&ms[0], c->ev[0], c->ev[1]));
    HIPCHK(hipEventElapsedTime(&ms[1], c->ev[1], c->ev[2]));
    // a chunked run's graph replays interleave the NMPC and PI launches: the
    // first span holds both and there is no separate PI time
    if (c->n_chunks > 1) ms[1] = -1.0f;
    HIPCHK(hipEventElapsedTime(&ms[2], c->ev[2], c->ev[3]));
    ms[3] = 0.0f;
    if (c->grad_ran) HIPCHK(hipEventElapsedTime(&ms[3], c->ev[4], c->ev[5]));
    return MC_CL_OK;
}

int mc_cl_tune(mc_cl_ctx* c, void* hip_stream, int32_t trial_intervals, mc_cl_tune_result* r) {
    if (!c || !r || trial_intervals < 1) return MC_CL_EINVAL;
    HIPCHK(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)hip_stream;
    std::memset(r, 0, sizeof(*r));
    static const int kSpw[MC_CL_TUNE_NSPW] = {4, 8, 16, 32, 64};
    // short segments keep the reverse pass's sub-step tape (C Ns 6 doubles
    // per lane) in the caches between its write and its read back (c2:
    // reverse pass 33.8 ms at C = 2 against 37.0 ms at C = 10); longer ones
    // only save checkpoint memory
    static const int kCk[MC_CL_TUNE_NCK] = {2, 5, 10, 25, 50};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        g_hip_error = "hipEventCreate failed";
        return MC_CL_EHIP;
    }
    auto timed = [&](auto&& launches, float& ms) -> int {
        HIPCHK(hipEventRecord(e0, st));
        const int rc = launches();
        if (rc != MC_CL_OK) return rc;
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        return MC_CL_OK;
    };
    int rc = MC_CL_OK;
    // NMPC: the campaign's own samples, cut to the first trial_intervals
    // intervals, for every candidate number of samples per wavefront
    DevParams dt = c->dp;
    dt.L_cap = trial_intervals;
    const Outs out{c->d_phi, c->d_flops, c->d_cnt, c->d_hash, nullptr, nullptr, nullptr, c->S};
    r->n_classes = (int32_t)c->classes.size();
    for (size_t k = 0; k < c->classes.size() && rc == MC_CL_OK; ++k) {
        NmpcClass& nc = c->classes[k];
        r->nmax[k] = nc.nmax;
        if (c->prm.nlp_form == 1) {
            // one sample per wavefront: nothing to choose
            for (int j = 0; j < MC_CL_TUNE_NSPW; ++j) r->nmpc_ms[k][j] = -1.0f;
            r->spw[k] = nc.spw;
            continue;
        }
        float best = INFINITY;
        int bspw = nc.spw;
        for (int j = 0; j < MC_CL_TUNE_NSPW && rc == MC_CL_OK; ++j) {
            const int cand = balanced_spw(nc.count, kSpw[j], nc.slots_full);
            if ((rc = plan_class(c, nc, cand)) != MC_CL_OK) break;
            float ms = 0.0f;
            rc = timed([&]() -> int {
                hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, c->d_queue + k, 1, 0);
                HIPCHK(hipGetLastError());
                NmpcWork wk{nc.d_pos, nc.count, nc.spw, nc.groups, c->d_queue + k, nullptr,
                            nc.d_tiles, nc.d_xs, nc.d_W, nc.tile_stride, nc.xs_stride,
                            nc.w_stride};
                HIPCHK(dispatch_nmpc(nc.nmax, c->prm.grad_mode, c->prm.model_nx, dt, wk, out,
                                     nc.slots, st));
                return MC_CL_OK;
            }, ms);
            r->nmpc_ms[k][j] = ms;
            if (rc == MC_CL_OK && ms < best) {
                best = ms;
                bspw = cand;
            }
        }
        if (rc == MC_CL_OK) rc = plan_class(c, nc, bspw);
        r->spw[k] = nc.spw;
    }
    // PI gradient: forward pass with checkpoints plus reverse pass, whole
    // campaign, for every candidate checkpoint interval up to the length
    if (rc == MC_CL_OK && c->prm.want_grad && c->n_pi) {
        float best = INFINITY;
        int bC = c->ckC;
        for (int j = 0; j < MC_CL_TUNE_NCK && rc == MC_CL_OK; ++j) {
            r->grad_ms[j] = -1.0f;
            if (j > 0 && kCk[j] > std::max(c->Lmax, 1)) continue;
            if ((rc = size_ckpt(c, kCk[j])) != MC_CL_OK) break;
            float ms = 0.0f;
            rc = timed([&]() -> int {
                HIPCHK(launch_pi(pi_k_of(c, c->n_pi), c->n_pi, st, c->dp, c->d_pos_pi, c->n_pi,
                                 out, c->d_ck, nullptr, (int64_t)0));
                HIPCHK(launch_pi_reverse(pi_k_of(c, c->n_pi), st, c->dp, c->d_pos_pi, c->n_pi,
                                         c->d_ck, c->d_tape, c->d_ivtape, c->d_gk));
                return MC_CL_OK;
            }, ms);
            r->grad_ms[j] = ms;
            if (rc == MC_CL_OK && ms < best) {
                best = ms;
                bC = kCk[j];
            }
        }
        if (rc == MC_CL_OK) rc = size_ckpt(c, bC);
        r->ckpt_interval = c->ckC;
    }
    // PI: lanes per sample, the whole PI pass (with the reverse pass at the
    // chosen C when the gradient is wanted) at each candidate; the results
    // are bitwise the same for every lane count
    if (rc == MC_CL_OK && c->n_pi) {
        static const int kK[MC_CL_TUNE_NPIK] = {1, 2, 4};
        const bool grad = c->prm.want_grad && c->d_ck;
        float best = INFINITY;
        int bk = pi_lanes(c->n_pi, c->n_cu);
        for (int j = 0; j < MC_CL_TUNE_NPIK && rc == MC_CL_OK; ++j) {
            float ms = 0.0f;
            rc = timed([&]() -> int {
                HIPCHK(launch_pi(kK[j], c->n_pi, st, c->dp, c->d_pos_pi, c->n_pi, out,
                                 grad ? c->d_ck : nullptr, nullptr, (int64_t)0));
                if (grad)
                    HIPCHK(launch_pi_reverse(kK[j], st, c->dp, c->d_pos_pi, c->n_pi, c->d_ck,
                                             c->d_tape, c->d_ivtape, c->d_gk));
                return MC_CL_OK;
            }, ms);
            r->pi_ms[j] = ms;
            if (rc == MC_CL_OK && ms < best) {
                best = ms;
                bk = kK[j];
            }
        }
        if (rc == MC_CL_OK) c->pi_k = bk;
        r->pi_lanes = bk;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the trial launches overwrote the outputs; the run graph holds the old
    // launch shape
    c->drop_graph();
    set_chunk_plan(c);
    c->ran = false;
    c->grad_ran = false;
    return rc;
}

int mc_cl_stream_create(int32_t n_cu, void** stream) {
    if (!stream) return MC_CL_EINVAL;
    *stream = nullptr;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    const int total = prop.multiProcessorCount;
    const int n = (n_cu <= 0 || n_cu > total) ? total : n_cu;
    std::vector<uint32_t> mask((size_t)(total + 31) / 32, 0u);
    for (int k = 0; k < n; ++k) mask[(size_t)k / 32] |= 1u << (k % 32);
    hipStream_t st = nullptr;
    HIPCHK(hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()));
    *stream = (void*)st;
    return MC_CL_OK;
}

int mc_cl_stream_destroy(void* stream) {
    if (!stream) return MC_CL_EINVAL;
    HIPCHK(hipStreamDestroy((hipStream_t)stream));
    return MC_CL_OK;
}

int mc_cl_workspace_size(const mc_cl_params* p, size_t* bytes) {
    if (!p || !bytes) return MC_CL_EINVAL;
    *bytes = 0;
    mc_cl_params q = *p;
    q.workspace = nullptr;
    q.workspace_size = 0;
    mc_cl_ctx* c = nullptr;
    const int rc = mc_cl_create(&q, &c);
    if (rc != MC_CL_OK) return rc;
    *bytes = c->bytes_aligned;
    mc_cl_destroy(c);
    return MC_CL_OK;
}

int mc_cl_run_static(const mc_cl_params* p, void* hip_stream, const mc_cl_outputs* o) {
    if (!o || !o->phi) return MC_CL_EINVAL;
    int rc = validate(p);
    if (rc != MC_CL_OK) return rc;
    if (o->traj_z || o->traj_u || o->traj_xhat || p->want_grad || p->chunk_samples > 0 ||
        p->sample_ids || p->kind || p->horizon || p->lengths || p->nlp_form != 0)
        return MC_CL_EUNSUPPORTED;
    const int64_t S = p->n_samples;
    // scratch layout (256-byte aligned pieces): per-sample kind, N, L,
    // positions, work, counters and hashes (the last two only when the
    // caller does not take them), queue counters, then the wavefront
    // slots' NMPC workspaces
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_plan = 3 * al((size_t)S * 4);
    const size_t b_pos = al((size_t)S * 8), b_fl = al((size_t)S * 8);
    const size_t b_cnt = o->counters ? 0 : al((size_t)C_NCNT * S * 4);
    const size_t b_hash = o->ashash ? 0 : al((size_t)S * 8);
    const size_t b_ctl = 256;
    const size_t fixed = b_plan + b_pos + b_fl + b_cnt + b_hash + b_ctl;
    int nmax_hi = nmax_class(p->N);
    for (int j = 0; j < p->n_horizon_choices; ++j)
        nmax_hi = std::max(nmax_hi, nmax_class(p->horizon_choices[j]));
    const int rw = p->model_nx == 3 ? rec_width<3>() : rec_width<1>();
    auto slot_bytes = [&](int nmax, int spw) {
        return al((size_t)V_COUNT * nmax * 64 * 8) + al((size_t)rw * nmax * 64 * 8) +
               al((size_t)spw * nmax * nmax * 8);
    };
    // the campaign must fit with at least one wavefront slot of one sample
    if (fixed + slot_bytes(nmax_hi, 1) > (size_t)MC_CL_STATIC_SCRATCH_BYTES) return MC_CL_EINVAL;

    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    if ((rc = scratch_ptr(dev, &base)) != MC_CL_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    unsigned char* q = base;
    auto take = [&](size_t b) { unsigned char* r = q; q += b; return r; };
    int32_t* d_kind = (int32_t*)take(al((size_t)S * 4));
    int32_t* d_N = (int32_t*)take(al((size_t)S * 4));
    int32_t* d_L = (int32_t*)take(al((size_t)S * 4));
    int64_t* d_pos = (int64_t*)take(b_pos);
    double* d_flops = (double*)take(b_fl);
    int32_t* d_cnt = o->counters ? o->counters : (int32_t*)take(b_cnt);
    uint64_t* d_hash = o->ashash ? o->ashash : (uint64_t*)take(b_hash);
    int* d_ctl = (int*)take(b_ctl);   // [0..3] queues, [4..7] list lengths
    unsigned char* ws = q;
    const size_t ws_bytes = (size_t)MC_CL_STATIC_SCRATCH_BYTES - (size_t)(q - base);

    const DevParams dp = to_dev(*p);
    hipLaunchKernelGGL(plan_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, dp, S,
                       d_kind, d_N, d_L);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(bucket_kernel, dim3(1), dim3(1024), 0, st, d_kind, d_N, S, d_pos, d_ctl + 4);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, st, d_ctl, 4, 0);
    HIPCHK(hipGetLastError());
    int counts[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(counts, d_ctl + 4, sizeof(counts), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));

    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    int n_cu = prop.multiProcessorCount;
    if (p->cu_limit > 0 && p->cu_limit < n_cu) n_cu = p->cu_limit;
    const Outs out{o->phi, d_flops, d_cnt, d_hash, nullptr, nullptr, nullptr, S};
    static const int nmaxs[3] = {16, 32, 64};
    int64_t off = 0;
    // horizon classes one after another on the stream, each using the whole
    // workspace region for its wavefront slots
    for (int k = 0; k < 3; ++k) {
        const int64_t count = counts[k];
        if (count == 0) continue;
        const int nmax = nmaxs[k];
        const int slots_full = blocks_per_cu(nmax, p->grad_mode, p->model_nx) * n_cu;
        int nmax_in_class = 1;
        if (p->n_horizon_choices > 0) {
            for (int j = 0; j < p->n_horizon_choices; ++j)
                if (nmax_class(p->horizon_choices[j]) == nmax)
                    nmax_in_class = std::max(nmax_in_class, p->horizon_choices[j]);
        } else {
            nmax_in_class = p->N;
        }
        int spw = p->samples_per_wave > 0
                      ? p->samples_per_wave
                      : balanced_spw(count, choose_spw(count, nmax_in_class, slots_full), slots_full);
        int64_t groups = (count + spw - 1) / spw;
        int64_t slots = std::min<int64_t>(groups, slots_full);
        slots = std::min<int64_t>(slots, (int64_t)(ws_bytes / slot_bytes(nmax, spw)));
        while (slots < 1 && spw > 1) {
            spw = std::max(1, spw / 2);
            groups = (count + spw - 1) / spw;
            slots = std::min<int64_t>(std::min<int64_t>(groups, slots_full),
                                      (int64_t)(ws_bytes / slot_bytes(nmax, spw)));
        }
        if (slots < 1) return MC_CL_EINVAL;   // cannot happen after the size check above
        const int64_t tile_stride = (int64_t)V_COUNT * nmax * 64;
        const int64_t xs_stride = (int64_t)rw * nmax * 64;
        const int64_t w_stride = (int64_t)spw * nmax * nmax;
        // three regions; each rounded up is at most `slots` times its
        // rounded per-slot size, so they fit in slots * slot_bytes
        double* tiles = (double*)ws;
        double* xs = (double*)(ws + al((size_t)slots * tile_stride * 8));
        double* W = (double*)(ws + al((size_t)slots * tile_stride * 8) +
                              al((size_t)slots * xs_stride * 8));
        NmpcWork wk{d_pos + off, count, spw, (int)groups, d_ctl + k, nullptr, tiles, xs, W,
                    tile_stride, xs_stride, w_stride};
        HIPCHK(dispatch_nmpc(nmax, p->grad_mode, p->model_nx, dp, wk, out, (int)slots, st));
        off += count;
    }
    if (counts[3] > 0) {
        HIPCHK(launch_pi(pi_lanes((int64_t)counts[3], n_cu), (int64_t)counts[3], st, dp, d_pos + off,
                         (int64_t)counts[3], out, nullptr, nullptr, (int64_t)0));
    }
    return MC_CL_OK;
}

int mc_cl_plan(mc_cl_ctx* c, int32_t* out, int max_classes) {
    if (!c || !out) return MC_CL_EINVAL;
    int n = 0;
    for (const auto& k : c->classes) {
        if (n >= max_classes) break;
        out[n * 5 + 0] = k.nmax;
        out[n * 5 + 1] = (int32_t)k.count;
        out[n * 5 + 2] = c->prm.nlp_form == 1 ? 64 / k.nmax : k.spw;
        out[n * 5 + 3] = k.groups;
        out[n * 5 + 4] = k.slots;
        ++n;
    }
    return n;
}

}  // extern "C"
