// Exchange with the host heuristic (Sec. 3.4; the appendix program): count
// the current and the returned assignments of every chain, and keep, per
// formula, the B best of the 2B stacked rows (current first; a stable
// ascending sort of the counts, the last B rows kept, so equal counts favour
// the returned rows).  A kept row takes the variance average nu of the chain
// it came from ([nu; nu] stacked).
#include <hip/hip_runtime.h>

#include "hp_internal.hpp"

namespace hp {

constexpr int kCountThreads = 256;

// satisfied clauses of assignment `v` (state layout) for every work item
__global__ __launch_bounds__(kCountThreads) void count_kernel(const FormulaDev *__restrict__ fd,
                                                              const WorkItem *__restrict__ work,
                                                              const uint4 *__restrict__ rec, int B,
                                                              const uint8_t *__restrict__ v,
                                                              int32_t *__restrict__ counts) {
    __shared__ int s_part[kCountThreads / kWave];
    const WorkItem w = work[blockIdx.x];
    const FormulaDev f = fd[w.f];
    const uint8_t *vb = v + f.var_off * B + (int64_t)w.b * f.n;
    const uint4 *r = rec + f.clause_off;
    int cnt = 0;
    for (int c = threadIdx.x; c < f.c; c += blockDim.x) {
        const uint4 q = r[c];
        const uint32_t len = rec_len(q.w), negm = rec_negm(q.w);
        const uint32_t e[7] = {q.x & 0xffffu, q.x >> 16, q.y & 0xffffu, q.y >> 16,
                               q.z & 0xffffu, q.z >> 16, q.w & 0xffffu};
        uint32_t m = 0;
        for (uint32_t k = 0; k < len; ++k) m |= (uint32_t)(vb[e[k] & 0x7fffu] & 1u) << k;
        cnt += ((m ^ negm) & ((1u << len) - 1u)) != 0u;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) s_part[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int total = 0;
        for (int i = 0; i < (int)blockDim.x / kWave; ++i) total += s_part[i];
        counts[blockIdx.x] = total;
    }
}

// per formula: source row (0..2B-1) of each kept row
__global__ void select_kernel(const int32_t *__restrict__ cnt_cur, const int32_t *__restrict__ cnt_ret, int B,
                              int32_t *__restrict__ src) {
    const int f = blockIdx.x;
    const int32_t *a = cnt_cur + (int64_t)f * B, *r = cnt_ret + (int64_t)f * B;
    for (int j = threadIdx.x; j < 2 * B; j += blockDim.x) {
        const int32_t cj = j < B ? a[j] : r[j - B];
        int rank = 0;
        for (int k = 0; k < 2 * B; ++k) {
            const int32_t ck = k < B ? a[k] : r[k - B];
            rank += (ck < cj || (ck == cj && k < j)) ? 1 : 0;
        }
        if (rank >= B) src[(int64_t)f * B + (rank - B)] = j;
    }
}

// gathers the kept rows (v and nu) into the staging buffers
__global__ void gather_rows_kernel(const FormulaDev *__restrict__ fd, const WorkItem *__restrict__ work, int B,
                                   const int32_t *__restrict__ src, const uint8_t *__restrict__ v_cur,
                                   const uint8_t *__restrict__ v_ret, const unsigned char *__restrict__ nu,
                                   int nu_bytes, uint8_t *__restrict__ v_out, unsigned char *__restrict__ nu_out) {
    const WorkItem w = work[blockIdx.x];           // destination row (formula w.f, chain w.b)
    const FormulaDev f = fd[w.f];
    const int j = src[(int64_t)w.f * B + w.b];
    const int64_t base = f.var_off * B;
    const uint8_t *vs = (j < B ? v_cur + base + (int64_t)j * f.n : v_ret + base + (int64_t)(j - B) * f.n);
    const int64_t nu_src = (base + (int64_t)(j % B) * f.n) * nu_bytes;
    const int64_t dst = base + (int64_t)w.b * f.n;
    for (int i = threadIdx.x; i < f.n; i += blockDim.x) v_out[dst + i] = vs[i];
    for (int64_t i = threadIdx.x; i < (int64_t)f.n * nu_bytes; i += blockDim.x)
        nu_out[dst * nu_bytes + i] = nu[nu_src + i];
}

hipError_t launch_merge(Plan &p, const hp_state &st, const uint8_t *cand, hipStream_t s) {
    const size_t items = (size_t)p.F * p.B;
    const size_t vbytes = (size_t)p.total_vars * p.B;
    if (!p.d_mg_cnt) {
        hipError_t e = hipMalloc((void **)&p.d_mg_cnt, 3 * items * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc((void **)&p.d_mg_v, vbytes);
        if (e == hipSuccess) e = hipMalloc((void **)&p.d_mg_nu, vbytes * 8);
        if (e != hipSuccess) return e;
    }
    int32_t *cnt_cur = p.d_mg_cnt, *cnt_ret = p.d_mg_cnt + items, *src = p.d_mg_cnt + 2 * items;
    count_kernel<<<(unsigned)items, kCountThreads, 0, s>>>(p.d_fd, p.d_work_fb, p.d_rec, p.B, st.v, cnt_cur);
    count_kernel<<<(unsigned)items, kCountThreads, 0, s>>>(p.d_fd, p.d_work_fb, p.d_rec, p.B, cand, cnt_ret);
    select_kernel<<<p.F, 256, 0, s>>>(cnt_cur, cnt_ret, p.B, src);
    gather_rows_kernel<<<(unsigned)items, 256, 0, s>>>(p.d_fd, p.d_work_fb, p.B, src, st.v, cand,
                                                        reinterpret_cast<const unsigned char *>(st.nu), st.nu_bytes,
                                                        p.d_mg_v, p.d_mg_nu);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(st.v, p.d_mg_v, vbytes, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(st.nu, p.d_mg_nu, vbytes * st.nu_bytes, hipMemcpyDeviceToDevice, s);
    return e;
}

}  // namespace hp
