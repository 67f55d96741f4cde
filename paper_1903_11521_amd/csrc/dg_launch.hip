// Launchers of the element kernels for one polynomial degree (DG_DEGREE),
// both precisions.  Compiled once per supported degree.
#include <cstring>
#include <type_traits>

#include "dg_kernels.hip"
#include "dg_tables.h"

#ifndef DG_DEGREE
#error "DG_DEGREE must be defined"
#endif

namespace {

constexpr int N = DG_DEGREE;

inline unsigned wave_blocks(int64_t E) { return (unsigned)((E + dgk::EPW - 1) / dgk::EPW); }

inline unsigned flat_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename real, bool MIX>
struct Launch {
    static_assert(sizeof(dgk::StepItem<real>) == sizeof(DgItem), "StepItem layout");

    static hipError_t pack_star(int64_t E, const double *dense, void *packed, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL(dgk::k_pack_star<real>, dim3(flat_blocks(E * 81)), dim3(256), 0, s, E, dense,
                           (real *)packed);
        return hipGetLastError();
    }
    static hipError_t predictor(int64_t E, double dt, const void *Q, const void *star, void *T, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_predictor<N, real>), dim3(wave_blocks(E)), dim3(64), 0, s, E, (real)dt,
                           (const real *)Q, (const real *)star, (real *)T);
        return hipGetLastError();
    }
    static hipError_t time_integral(int64_t E, double dt, const void *T, void *I, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_time_integral<N, real>), dim3(flat_blocks(E * 9 * dgk::nb3(N))), dim3(256), 0,
                           s, E, dt, (const real *)T, (real *)I);
        return hipGetLastError();
    }
    static hipError_t volume(int64_t E, const void *I, const void *star, void *Q, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_volume<N, real>), dim3(wave_blocks(E)), dim3(64), 0, s, E, (const real *)I,
                           (const real *)star, (real *)Q);
        return hipGetLastError();
    }
    static hipError_t local_flux(int64_t E, const void *I, const double *Ap, void *Q, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_local_flux<N, MIX, real>), dim3(wave_blocks(E)), dim3(64), 0, s, E,
                           (const real *)I, Ap, (real *)Q);
        return hipGetLastError();
    }
    static hipError_t neighbour_flux(int64_t E, int64_t nI, const void *I, const int32_t *neigh,
                                     const uint8_t *fr, const double *Am, void *Q, hipStream_t s)
    {
        if (E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_neighbour_flux<N, MIX, real>), dim3(wave_blocks(E)), dim3(64), 0, s, E, nI,
                           (const real *)I, neigh, fr, Am, (real *)Q);
        return hipGetLastError();
    }
    static hipError_t step_predict(const DgItem &it, hipStream_t s)
    {
        if (it.E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_step_predict<N, MIX, real>), dim3(wave_blocks(it.E)), dim3(64), 0, s, it.E, it.dt,
                           (const real *)it.Q, (const real *)it.star, (real *)it.I, (real *)it.traces);
        return hipGetLastError();
    }
    static hipError_t step_correct(const DgItem &it, hipStream_t s)
    {
        if (it.E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_step_correct<N, MIX, real>), dim3(wave_blocks(it.E)), dim3(64), 0, s, it.E,
                           it.nI < it.E ? it.E : it.nI, (const real *)it.I, (const real *)it.traces, (const real *)it.star, it.Ap, it.Am,
                           it.neigh, it.face_rot, (real *)it.Q);
        return hipGetLastError();
    }
    // corrector of step n (traces of step n in it.traces) + predictor of step
    // n+1 (its traces to tr_out)
    static hipError_t step_fused(const DgItem &it, void *tr_out, hipStream_t s)
    {
        if (it.E == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_step_fused<N, MIX, real>), dim3(wave_blocks(it.E)), dim3(64), 0, s, it.E, it.dt,
                           (real *)it.I, (const real *)it.traces, (real *)tr_out, (const real *)it.star, it.Ap,
                           it.Am, it.neigh, it.face_rot, (real *)it.Q);
        return hipGetLastError();
    }
    static hipError_t batch_predict(const DgItem *items, const int32_t *block_item, int64_t nblocks, hipStream_t s)
    {
        if (nblocks == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_batch_predict<N, MIX, real>), dim3((unsigned)nblocks), dim3(64), 0, s,
                           (const dgk::StepItem<real> *)items, block_item);
        return hipGetLastError();
    }
    static hipError_t batch_correct(const DgItem *items, const int32_t *block_item, int64_t nblocks, hipStream_t s)
    {
        if (nblocks == 0) return hipSuccess;
        hipLaunchKernelGGL((dgk::k_batch_correct<N, MIX, real>), dim3((unsigned)nblocks), dim3(64), 0, s,
                           (const dgk::StepItem<real> *)items, block_item);
        return hipGetLastError();
    }
    static void fill(DgTable *t)
    {
        t->pack_star = pack_star;
        t->predictor = predictor;
        t->time_integral = time_integral;
        t->volume = volume;
        t->local_flux = local_flux;
        t->neighbour_flux = neighbour_flux;
        t->step_predict = step_predict;
        t->step_correct = step_correct;
        t->step_fused = step_fused;
        // fused launch slower than predictor + corrector from degree 4 on
        // (larger code and register footprint of the combined kernel)
        t->fuse_step = N <= 3;
        t->batch_predict = batch_predict;
        t->batch_correct = batch_correct;
    }
};

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

void DG_CAT(dg_table_, DG_DEGREE)(DgTable *fp64, DgTable *fp32, DgTable *mixed)
{
    Launch<double, false>::fill(fp64);
    Launch<float, false>::fill(fp32);
    // mixed form: FP32 storage and contractions; it differs from plain FP32
    // in the time-integral accumulation and the flux-solver products (FP64)
    Launch<float, false>::fill(mixed);
    mixed->local_flux = Launch<float, true>::local_flux;
    mixed->neighbour_flux = Launch<float, true>::neighbour_flux;
    mixed->step_predict = Launch<float, true>::step_predict;
    mixed->step_correct = Launch<float, true>::step_correct;
    mixed->step_fused = Launch<float, true>::step_fused;
    mixed->batch_predict = Launch<float, true>::batch_predict;
    mixed->batch_correct = Launch<float, true>::batch_correct;
}
