// Dataflow sweeps: all steps of the forward and backward passes of the sweeping
// preconditioner (paper Sec. 5 eq. (7), Sec. 6), and optionally the operator (I - S) that
// GMRES applies next (Sec. 4 eq. (5)), in one launch of persistent workgroups.
//
// A sweep step of the paper is a set of independent local scatterings whose inputs are the
// outputs of the previous step on the neighbouring subdomains.  Launching one kernel per step
// leaves the chip idle between steps; here every (stage, subdomain, right-hand side, row block)
// is a task.  Workgroups claim tasks from a ticket counter in a fixed topological order (steps
// in sweep order, then the next stage); a task first issues the loads of its 8 x L block of the
// dense scattering operator, which depend on no data, then waits until the completion counters
// of the tasks that produce its incoming data have reached their totals, then reads the data
// and finishes.  A task only ever waits for tasks with smaller tickets, which were claimed by
// workgroups that are running, so the launch completes whatever the number of resident
// workgroups.  Every wait is bounded: past spin_limit polls it sets the error flag and goes on,
// so every wave exits.
//
// Memory ordering without cache-wide fences: every interface datum that a task may read from
// another task of the same launch is written and read with agent-scope (device-coherent)
// accesses, so no L2 writeback or invalidation is needed.  The producing wavefront waits until
// its coherent stores have completed (s_waitcnt) before it increments the counter; the
// consumer polls the counter with coherent loads and only then, after a workgroup barrier,
// issues the coherent loads of the data.  The operator blocks (read-only) use ordinary loads.
#include "hbj_internal.h"

namespace {

constexpr int CG = 32;      // column groups (8 rows x 32 groups = 256 threads)

// device-coherent 128-bit accesses as two 64-bit agent-scope atomics
__device__ inline double2 ld_dev(const double2* p) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return mk(__longlong_as_double((long long)a), __longlong_as_double((long long)b));
}
__device__ inline void st_dev(double2* p, double2 v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  __hip_atomic_store(q, (unsigned long long)__double_as_longlong(v.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, (unsigned long long)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
constexpr int LMAX = 1024;  // local interface length limit

// branch-wise selection keeps the stage table in kernel-argument registers (a select by a
// runtime index goes through a private copy)
__device__ inline DfStage stage_of(const DfArgs& A, int i) {
  if (i == 0) return A.st[0];
  if (i == 1) return A.st[1];
  return A.st[2];
}

template <typename C, int KMAX>
__global__ __launch_bounds__(kTR * CG) void k_sweep_df(Geom g, const DfTask* __restrict__ tasks, int ntasks,
                                                       const FaceTab* __restrict__ ft, const C* __restrict__ T,
                                                       DfArgs A, int32_t* ctr, int32_t* ctr_next, int nctr,
                                                       int32_t* err, int spin_limit, int stall_task) {
  // the other counter region is zeroed here for the next launch (it is not used by this one)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nctr; i += gridDim.x * blockDim.x) ctr_next[i] = 0;
  __shared__ int s_ticket;
  __shared__ double2 gl[LMAX];
  __shared__ double2 red[kTR * CG / 64][kTR];
  const int L = local_if_len(g);
  const size_t per = t_per_sub(g);
  const int r = threadIdx.x % kTR, grp = threadIdx.x / kTR;
  int32_t* counters = ctr + 1;
  const int nslots = nctr - 1;
  for (;;) {
    // The loop is uniform by construction: the ticket goes through LDS and is read back as a
    // scalar, so the exit branch is a scalar branch and every wave runs every barrier once per
    // task.  (A loop whose exit the compiler must treat as divergent can be restructured so
    // that a subset of lanes repeats the barrier section without passing the ticket claim.)
    __syncthreads();  // the previous task no longer reads s_ticket, gl or red
    if (threadIdx.x == 0) s_ticket = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int ti = __builtin_amdgcn_readfirstlane(s_ticket);
    if (ti < 0 || ti >= ntasks) break;
    const DfTask* tp = tasks + ti;
    const int t_stage = tp->stage, t_s = tp->s, t_rhs = tp->rhs, t_rb = tp->rb, t_first = tp->first;
    const DfStage S = stage_of(A, t_stage);
    const FaceTab F = ft[t_s];
    // 1. operator rows (independent of the data)
    const C* Tb = T + (size_t)t_s * per + (size_t)t_rb * L * kTR + r;
    C v[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int col = grp + CG * k;
      v[k].x = 0;
      v[k].y = 0;
      if (col < L) v[k] = Tb[(size_t)col * kTR];
    }
    // 2. wait for the producers of the incoming data
    if (threadIdx.x == 0) {
      // one poll budget for all the task's waits; out-of-range entries count as failures
      const int ndep = min(max(tp->ndep, 0), kDfMaxDeps);
      int polls = 0;
      for (int d = 0; d < ndep; ++d) {
        const int q = tp->dep[d];
        if (q < 0 || q >= nslots) {
          __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        const int need = tp->need[d] + (ti == stall_task ? 1 : 0);
        bool gave_up = false;
        while (__hip_atomic_load(counters + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++polls > spin_limit) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gave_up = true;
            break;
          }
          // once any wait has given up, every other wait gives up too
          if ((polls & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            gave_up = true;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (gave_up) break;
      }
    }
    __syncthreads();
    // 3. incoming data of the subdomain (absent faces are zero)
    const size_t cb = (size_t)t_rhs * g.nif;
    for (int q = threadIdx.x; q < L; q += blockDim.x) {
      int f, ee;
      local_if_face(g, q, &f, &ee);
      const int o = pick4(F.in_off, f);
      const bool from_out = !t_first && ((S.out_read >> f) & 1);
      gl[q] = (o >= 0) ? ld_dev((from_out ? S.out : S.in) + cb + o + ee) : mk(0.0, 0.0);
    }
    __syncthreads();
    double2 acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int col = grp + CG * k;
      if (col < L) cfma(acc, to_d(v[k]), gl[col]);
    }
#pragma unroll
    for (int off = kTR; off < 64; off <<= 1) {
      acc.x += __shfl_xor(acc.x, off);
      acc.y += __shfl_xor(acc.y, off);
    }
    if ((threadIdx.x & 63) < kTR) red[threadIdx.x >> 6][r] = acc;
    __syncthreads();
    // 4. rows of the block (all in wavefront 0), then publish
    if (threadIdx.x < 64) {
      const int row = t_rb * kTR + (int)threadIdx.x;
      if (threadIdx.x < kTR && row < L) {
        int rf, re;
        local_if_face(g, row, &rf, &re);
        if ((S.mask >> rf) & 1) {
          const int oo = pick4(F.out_off, rf);
          if (oo >= 0) {
            double2 sum = red[0][r];
#pragma unroll
            for (int w = 1; w < kTR * CG / 64; ++w) sum = cadd(sum, red[w][r]);
            const size_t o = cb + oo + re;
            double2 b = ld_dev(S.base + o);
            b.x += S.sign * sum.x;
            b.y += S.sign * sum.y;
            st_dev(S.dst + o, b);
          }
          const int io = pick4(F.in_off, rf);
          if (S.copy && io >= 0) st_dev(S.dst + cb + io + re, ld_dev(S.in + cb + io + re));
        }
      }
      // the coherent stores complete before the counter moves
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_s_waitcnt(0);
      const int slot = tp->slot;
      if (threadIdx.x == 0 && slot >= 0 && slot < nslots)
        __hip_atomic_fetch_add(counters + slot, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename C>
const void* df_kernel(int L) {
  if (L <= 16 * CG) return (const void*)k_sweep_df<C, 16>;
  return (const void*)k_sweep_df<C, LMAX / CG>;
}

}  // namespace

int sweep_df_occupancy(int L, bool c64) {
  int n = 0;
  const void* k = c64 ? df_kernel<float2>(L) : df_kernel<double2>(L);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kTR * CG, 0) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <typename C>
hipError_t launch_sweep_df(const Geom& g, const DfTask* tasks, int ntasks, const FaceTab* ft, const C* T,
                           const DfArgs& A, int32_t* ctr, int32_t* ctr_next, int nctr, int32_t* err, int spin_limit,
                           int stall_task, int grid, hipStream_t st) {
  if (ntasks == 0) return hipSuccess;
  const int L = local_if_len(g);
  if (L > LMAX || grid <= 0) return hipErrorInvalidValue;
  if (L <= 16 * CG)
    hipLaunchKernelGGL((k_sweep_df<C, 16>), dim3(grid), dim3(kTR * CG), 0, st, g, tasks, ntasks, ft, T, A, ctr,
                       ctr_next, nctr, err, spin_limit, stall_task);
  else
    hipLaunchKernelGGL((k_sweep_df<C, LMAX / CG>), dim3(grid), dim3(kTR * CG), 0, st, g, tasks, ntasks, ft, T, A,
                       ctr, ctr_next, nctr, err, spin_limit, stall_task);
  return hipGetLastError();
}

template hipError_t launch_sweep_df<double2>(const Geom&, const DfTask*, int, const FaceTab*, const double2*,
                                             const DfArgs&, int32_t*, int32_t*, int, int32_t*, int, int, int, hipStream_t);
template hipError_t launch_sweep_df<float2>(const Geom&, const DfTask*, int, const FaceTab*, const float2*,
                                            const DfArgs&, int32_t*, int32_t*, int, int32_t*, int, int, int, hipStream_t);
