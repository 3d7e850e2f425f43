// cells.hip -- prior cells of the new state in a kernel of their own (section
// 2.1: the moving prior is the mean weight of the particles in a cell of the
// integrals of motion).  Used where the fused step kernel cannot hold the cell
// sums next to the observables in LDS (the learned prior's judge grid): that
// kernel then observes without cells, and this one decides each particle's cell
// (FP32 with a guard band, FP64 inside it), stores its tag and sums weights and
// counts per cell into the cell columns of the same partial slots, with the
// same block-to-slot assignment.
#include "particle.h"
#include "forms.h"

namespace m2m {

template <int POT>
__global__ void __launch_bounds__(1024) cells_kernel(StepArgs<float, float> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int failed = *a.flag;
    const int NC = a.cells.ncell, JP = a.jpad;
    double* csum = reinterpret_cast<double*>(smem);                  // NC
    float2* et = reinterpret_cast<float2*>(csum + NC);               // uniform-E Lc table
    unsigned* ccnt = reinterpret_cast<unsigned*>(et + kLcE);         // NC
    const int nt = blockDim.x, tid = threadIdx.x;
    const int t0 = ro(a.block_tile0, blockIdx.x), t1 = ro(a.block_tile0, blockIdx.x + 1);
    int slot = ro(a.block_slot0, blockIdx.x) - 1, cur = -1;
    Pot<float> pot{};
    float Emin = 0.0f, sE = 0.0f;
    CellGuard cg{};
    if (failed) return;
    const uint32_t rb = uint32_t(a.stride * sizeof(float));
    uint16_t* tags = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(a.out) + 7 * (size_t)rb) +
                     (size_t)a.cellrow * a.stride;
    for (int t = t0; t <= t1; ++t) {
        const int m = t < t1 ? ro(a.tile_model, t) : -2;
        if (m != cur) {
            if (cur >= 0) {
                // the finished model's cell columns of its partial slot
                __syncthreads();
                float* dst = a.part + ro(a.slot_base, slot);
                const int64_t cs = ro(a.slot_stride, slot);
                for (int c = tid; c < NC; c += nt) {
                    const int j0 = JP + 2 * c, j1 = j0 + 1;
                    dst[(j0 / kFinCols) * cs + j0 % kFinCols] = float(csum[c]);
                    dst[(j1 / kFinCols) * cs + j1 % kFinCols] = float(ccnt[c]);
                }
            }
            if (m < 0) break;
            cur = m;
            ++slot;
            pot = ro(a.pots, m);
            Emin = ro(a.erange, 2 * m);
            sE = float(a.cells.n0) / (ro(a.erange, 2 * m + 1) - Emin);
            cg = cell_guard(Emin, ro(a.erange, 2 * m + 1), sE);
            __syncthreads();
            for (int c = tid; c < NC; c += nt) { csum[c] = 0.0; ccnt[c] = 0u; }
            for (int i = tid; i < kLcE; i += nt)
                et[i] = make_float2(a.lcetab[2 * ((size_t)m * kLcE + i)], a.lcetab[2 * ((size_t)m * kLcE + i) + 1]);
            __syncthreads();
        }
        const int64_t p0 = ro(a.tile_p0, t);
        const int cnt = ro(a.tile_cnt, t);
        for (int i = tid; i < cnt; i += nt) {
            const int64_t p = p0 + i;
            const uint32_t o = uint32_t(p) * 4u;
            const float x = ld_at<float>(a.out, o), y = ld_at<float>(a.out, o + rb), z = ld_at<float>(a.out, o + 2 * rb);
            const float vx = ld_at<float>(a.out, o + 3 * rb), vy = ld_at<float>(a.out, o + 4 * rb);
            const float vz = ld_at<float>(a.out, o + 5 * rb), w = ld_at<float>(a.out, o + 6 * rb);
            float phi, ax, ay, az;
            potential<POT, float>(pot, x, y, z, phi, ax, ay, az);
            const float KE = 0.5f * (vx * vx + vy * vy + vz * vz);
            int cell;
            if (cell_fast<POT>(pot, et, a.cells, Emin, sE, cg, KE, phi, x, y, z, vx, vy, vz, cell) != 0u) {
                const Exact* ex = a.ex;
                const Pot<double>& pd = ex->pots[m];
                cell = prior_cell_seeded<POT>(pd, ex->lctab + pd.lc_off, ex->rce + (size_t)m * kLcE, double(pot.lcE0),
                                              double(pot.lcEinv), a.cells, ex->erange[2 * m], ex->erange[2 * m + 1],
                                              double(x), double(y), double(z), double(vx), double(vy), double(vz));
            }
            tags[p] = (uint16_t)cell;
            atomicAdd(&csum[cell], double(w));
            atomicAdd(&ccnt[cell], 1u);
        }
    }
}

hipError_t launch_cells(const StepArgs<float, float>& a, int pot_kind, int blocks, size_t lds, hipStream_t s) {
    switch (pot_kind) {
        case 0: hipLaunchKernelGGL(cells_kernel<0>, dim3(blocks), dim3(1024), lds, s, a); break;
        case 1: hipLaunchKernelGGL(cells_kernel<1>, dim3(blocks), dim3(1024), lds, s, a); break;
        default: hipLaunchKernelGGL(cells_kernel<2>, dim3(blocks), dim3(1024), lds, s, a); break;
    }
    return hipGetLastError();
}

hipError_t set_cells_lds_limit(size_t lds) {
    for (const void* f : {(const void*)cells_kernel<0>, (const void*)cells_kernel<1>, (const void*)cells_kernel<2>}) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace m2m
