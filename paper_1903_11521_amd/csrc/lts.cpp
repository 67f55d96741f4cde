// Clustered local time stepping of rate 2 (the LTS of Sec. 6.4 and Table
// tab:loh1): cluster c steps with dt_c = 2^c dt0, face neighbours differ by
// at most one cluster, and the neighbour term of an element's step (Eq.
// seissol:correction_neigh) takes each neighbour's time integral over the
// element's own step interval:
//   same cluster:    the neighbour's step integral;
//   larger cluster:  the neighbour's Taylor expansion integrated over the
//                    half of its step that the element's step covers;
//   smaller cluster: the sum of the neighbour's two step integrals.
// One cycle is 2^(C-1) ticks of dt0.  At each tick the clusters whose step
// starts there run their predictor; then the clusters whose step ends at
// the next tick are corrected.  Elements are numbered cluster by cluster.
//
// Every cluster runs on the step kernels.  The neighbour term reads face
// traces (R^T of the integral, linear in it), so a cluster's trace array
// holds its own elements' slots followed by ghost slots, one per neighbour
// in another cluster, and a cluster-relative neighbour table points at
// them.  Before a cluster's corrector its ghost slots are filled:
//   larger neighbour: the predictor run a second time with dt/2 gives the
//                     traces of the first half of its step (the Taylor
//                     expansion does not depend on dt); the second half is
//                     the full step's traces minus the first half's;
//   smaller neighbour: a trace buffer that sums its two steps' traces.
// The second predictor runs from the cluster's first element with a
// neighbour one cluster down; numbering those elements last keeps it short
// (any order within a cluster gives the same result).
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "dg_internal.h"
#include "lts_internal.h"

struct dg_lts {
    const dg_plan *plan = nullptr;
    int64_t E = 0;
    int C = 0;
    double dt0 = 0.0;
    size_t elem = 8;
    int PB = 0, TB = 0;                     // values per DOF block and per trace slot
    std::vector<int64_t> start;             // C + 1 cluster offsets
    std::vector<int64_t> tstart;            // per cluster: first element with a neighbour one cluster down
    std::vector<int64_t> region;            // C + 1 offsets of the clusters' trace regions (own + ghost slots)
    std::vector<int64_t> nghost;
    void *I = nullptr, *IH = nullptr;       // [E][PB] step and half-step integrals
    void *TR = nullptr;                     // trace regions, region[C] slots
    void *TRH = nullptr, *TRB = nullptr;    // [E][TB] half-step traces, trace buffer
    int32_t *neigh_rel = nullptr;           // [E][4] cluster-relative neighbour table
    void *lists = nullptr;                  // device: ghost ids, ghost kinds and buffer ids of all clusters
    std::vector<const int32_t *> gids, bids;
    std::vector<const int8_t *> gkind;
    std::vector<int64_t> nbuf;

    ~dg_lts()
    {
        for (void *p : {I, IH, TR, TRH, TRB, (void *)neigh_rel, lists})
            if (p) (void)hipFree(p);
    }
};

namespace {

int fail(int code, const char *fmt, long long a = 0, long long b = 0, long long c = 0)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, a, b, c);
    return dg_set_error(code, buf);
}

int hip_fail(hipError_t e, const char *where)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
    return dg_set_error(DG_EHIP, buf);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" {

int dg_lts_create(const dg_plan *plan, int64_t E, const int32_t *cluster, const int32_t *neigh, double dt0,
                  dg_lts **out)
{
    if (!out) return fail(DG_EINVAL, "dg_lts_create: null output pointer");
    *out = nullptr;
    if (!plan) return fail(DG_EINVAL, "dg_lts_create: null plan");
    if (plan->prec == DG_BF16X3 || !plan->tab.step_predict || !plan->tab.step_correct)
        return fail(DG_EUNSUPPORTED, "dg_lts_create: not available for this precision (split-BF16 form)");
    if (E < 0 || E > 0x7fffffff) return fail(DG_EINVAL, "dg_lts_create: element count %lld out of range", E);
    if (E > 0 && (!cluster || !neigh)) return fail(DG_EINVAL, "dg_lts_create: null cluster or neighbour table");
    if (!(dt0 > 0.0) || !std::isfinite(dt0)) return fail(DG_EINVAL, "dg_lts_create: dt0 must be positive and finite");
    int C = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int c = cluster[e];
        if (c < 0 || c >= DG_LTS_MAX_CLUSTERS)
            return fail(DG_EINVAL, "dg_lts_create: cluster %lld of element %lld outside [0, %lld)", c, e,
                        DG_LTS_MAX_CLUSTERS);
        if (e > 0 && c < cluster[e - 1])
            return fail(DG_EINVAL, "dg_lts_create: elements not numbered cluster by cluster (element %lld)", e);
        if (c + 1 > C) C = c + 1;
    }
    for (int64_t e = 0; e < E; ++e)
        for (int s = 0; s < 4; ++s) {
            const int32_t v = neigh[e * 4 + s];
            if (v < -1 || v >= E)
                return fail(DG_EINVAL, "dg_lts_create: neighbour %lld of element %lld outside [-1, E)", v, e);
            if (v >= 0 && std::abs(cluster[v] - cluster[e]) > 1)
                return fail(DG_EINVAL, "dg_lts_create: neighbours %lld and %lld differ by more than one cluster",
                            e, v);
        }
    dg_lts *L = new (std::nothrow) dg_lts;
    if (!L) return fail(DG_ENOMEM, "dg_lts_create: out of host memory");
    L->plan = plan;
    L->E = E;
    L->C = C;
    L->dt0 = dt0;
    L->elem = plan->prec == DG_FP64 ? 8 : 4;
    L->PB = 9 * plan->B;
    L->TB = 4 * 9 * plan->Bf;
    L->start.assign((size_t)C + 1, E);
    for (int64_t e = E - 1; e >= 0; --e) L->start[(size_t)cluster[e]] = e;
    for (int c = C - 1; c >= 0; --c)
        if (L->start[(size_t)c] > L->start[(size_t)c + 1]) L->start[(size_t)c] = L->start[(size_t)c + 1];
    // per cluster: ghosts (neighbours in other clusters, each once, with
    // kind 1 = one up, 2 = one down), elements with a neighbour one up (their
    // traces are buffered), the first element with a neighbour one down; the
    // cluster-relative neighbour table
    std::vector<std::vector<int32_t>> gi((size_t)C), bi((size_t)C);
    std::vector<std::vector<int8_t>> gk((size_t)C);
    std::vector<int64_t> slot((size_t)E, -1), mark((size_t)E, -1);
    std::vector<int32_t> nrel((size_t)E * 4, -1);
    L->tstart.assign((size_t)C, 0);
    L->nghost.assign((size_t)C, 0);
    for (int c = 0; c < C; ++c) {
        const int64_t s0 = L->start[(size_t)c], s1 = L->start[(size_t)c + 1];
        int64_t first_down = s1;
        for (int64_t e = s0; e < s1; ++e) {
            bool up = false;
            for (int s = 0; s < 4; ++s) {
                const int32_t v = neigh[e * 4 + s];
                if (v < 0) continue;
                const int dc = cluster[v] - c;
                if (dc == 0) {
                    nrel[(size_t)(e * 4 + s)] = (int32_t)(v - s0);
                    continue;
                }
                if (dc == 1) up = true;
                if (dc == -1 && first_down == s1) first_down = e;
                if (mark[(size_t)v] != c) {
                    mark[(size_t)v] = c;
                    slot[(size_t)v] = (int64_t)gi[(size_t)c].size();
                    gi[(size_t)c].push_back(v);
                    gk[(size_t)c].push_back((int8_t)(dc == 1 ? 1 : 2));
                }
                nrel[(size_t)(e * 4 + s)] = (int32_t)((s1 - s0) + slot[(size_t)v]);
            }
            if (up) bi[(size_t)c].push_back((int32_t)e);
        }
        L->tstart[(size_t)c] = first_down;
        L->nghost[(size_t)c] = (int64_t)gi[(size_t)c].size();
    }
    L->region.assign((size_t)C + 1, 0);
    for (int c = 0; c < C; ++c)
        L->region[(size_t)c + 1] = L->region[(size_t)c] + (L->start[(size_t)c + 1] - L->start[(size_t)c]) +
                                   L->nghost[(size_t)c];
    size_t n32 = 0, n8 = 0;
    for (int c = 0; c < C; ++c) n32 += gi[(size_t)c].size() + bi[(size_t)c].size(), n8 += gk[(size_t)c].size();
    const size_t pe = (size_t)L->PB * L->elem, te = (size_t)L->TB * L->elem;
    hipError_t h = hipSuccess;
    if (E > 0) {
        if ((h = hipMalloc(&L->I, (size_t)E * pe)) == hipSuccess &&
            (h = hipMalloc(&L->IH, (size_t)E * pe)) == hipSuccess &&
            (h = hipMalloc(&L->TR, (size_t)L->region[(size_t)C] * te)) == hipSuccess &&
            (h = hipMalloc(&L->TRH, (size_t)E * te)) == hipSuccess &&
            (h = hipMalloc(&L->TRB, (size_t)E * te)) == hipSuccess &&
            (h = hipMalloc((void **)&L->neigh_rel, (size_t)E * 16)) == hipSuccess)
            h = hipMalloc(&L->lists, n32 * 4 + n8 + 16);
        if (h == hipSuccess) h = hipMemcpy(L->neigh_rel, nrel.data(), nrel.size() * 4, hipMemcpyHostToDevice);
    }
    if (h != hipSuccess) {
        delete L;
        return h == hipErrorOutOfMemory ? fail(DG_ENOMEM, "dg_lts_create: out of device memory")
                                        : hip_fail(h, "dg_lts_create");
    }
    std::vector<unsigned char> blob(n32 * 4 + n8);
    size_t off32 = 0, off8 = n32 * 4;
    L->gids.resize((size_t)C);
    L->bids.resize((size_t)C);
    L->gkind.resize((size_t)C);
    L->nbuf.resize((size_t)C);
    unsigned char *dev = static_cast<unsigned char *>(L->lists);
    for (int c = 0; c < C; ++c) {
        const auto &g = gi[(size_t)c], &b = bi[(size_t)c];
        const auto &k = gk[(size_t)c];
        L->nbuf[(size_t)c] = (int64_t)b.size();
        L->gids[(size_t)c] = reinterpret_cast<const int32_t *>(dev + off32);
        if (!g.empty()) std::memcpy(blob.data() + off32, g.data(), g.size() * 4);
        off32 += g.size() * 4;
        L->bids[(size_t)c] = reinterpret_cast<const int32_t *>(dev + off32);
        if (!b.empty()) std::memcpy(blob.data() + off32, b.data(), b.size() * 4);
        off32 += b.size() * 4;
        L->gkind[(size_t)c] = reinterpret_cast<const int8_t *>(dev + off8);
        if (!k.empty()) std::memcpy(blob.data() + off8, k.data(), k.size());
        off8 += k.size();
    }
    if (!blob.empty() && (h = hipMemcpy(L->lists, blob.data(), blob.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        delete L;
        return hip_fail(h, "dg_lts_create");
    }
    *out = L;
    return DG_OK;
}

int dg_lts_clusters(const dg_lts *lts, int *n_clusters, int64_t *updates_per_cycle)
{
    if (!lts) return fail(DG_EINVAL, "dg_lts_clusters: null handle");
    if (n_clusters) *n_clusters = lts->C;
    if (updates_per_cycle) {
        int64_t u = 0;
        for (int c = 0; c < lts->C; ++c)
            u += (lts->start[(size_t)c + 1] - lts->start[(size_t)c]) << (lts->C - 1 - c);
        *updates_per_cycle = u;
    }
    return DG_OK;
}

int dg_lts_advance(dg_lts *lts, int n_cycles, void *Q, const void *star_packed, const double *Aplus,
                   const double *Aminus, const int32_t *neigh, const uint8_t *face_rot, hipStream_t s)
{
    if (!lts) return fail(DG_EINVAL, "dg_lts_advance: null handle");
    if (n_cycles < 0) return fail(DG_EINVAL, "dg_lts_advance: negative cycle count %lld", n_cycles);
    if (lts->E == 0 || n_cycles == 0) return DG_OK;
    const void *ptrs[] = {Q, star_packed, Aplus, Aminus, neigh, face_rot};
    for (const void *p : ptrs)
        if (!p || !aligned16(p)) return fail(DG_EINVAL, "dg_lts_advance: null or not 16-byte aligned array");
    // the neighbour table itself is read at creation (host copy); the handle
    // holds the cluster-relative form the kernels use
    const DgTable &t = lts->plan->tab;
    const bool fp64 = lts->elem == 8;
    const int C = lts->C, TB = lts->TB;
    const size_t qe = (size_t)lts->PB * lts->elem, te = (size_t)TB * lts->elem, se = 81 * lts->elem,
                 ae = 4 * 81 * 8;
    auto at = [](const void *p, int64_t e, size_t stride) {
        return const_cast<char *>(static_cast<const char *>(p)) + (size_t)e * stride;
    };
    // base pointer p with p + v * te = element v's own slot in cluster c's
    // region (region[c] >= start[c], so p lies inside the array)
    auto own_base = [&](int c) { return at(lts->TR, lts->region[(size_t)c] - lts->start[(size_t)c], te); };
    auto item = [&](int c, int64_t e0, int64_t e1, double dt, void *I, void *traces) {
        DgItem it;
        it.E = e1 - e0;
        it.dt = dt;
        it.Q = at(Q, e0, qe);
        it.I = at(I, e0, qe);
        it.traces = traces;
        it.star = at(star_packed, e0, se);
        it.Ap = reinterpret_cast<const double *>(at(Aplus, e0, ae));
        it.Am = reinterpret_cast<const double *>(at(Aminus, e0, ae));
        it.neigh = lts->neigh_rel + e0 * 4;
        it.face_rot = reinterpret_cast<const uint8_t *>(at(face_rot, e0, 4));
        it.first_block = 0;
        it.nI = it.E + (c >= 0 ? lts->nghost[(size_t)c] : 0);
        return it;
    };
    const int64_t ticks = int64_t(1) << (C - 1);
    hipError_t h = hipSuccess;
#define LTS_HIP(call)                                                      \
    do {                                                                   \
        if ((h = (call)) != hipSuccess) return hip_fail(h, "dg_lts_advance"); \
    } while (0)
    for (int cyc = 0; cyc < n_cycles; ++cyc) {
        for (int64_t tau = 0; tau < ticks; ++tau) {
            for (int c = 0; c < C; ++c) {
                const int64_t s0 = lts->start[(size_t)c], s1 = lts->start[(size_t)c + 1];
                if (s1 == s0 || tau % (int64_t(1) << c) != 0) continue;
                const double dtc = std::ldexp(lts->dt0, c);
                LTS_HIP(t.step_predict(item(c, s0, s1, dtc, lts->I, at(lts->TR, lts->region[(size_t)c], te)), s));
                const int64_t t0 = lts->tstart[(size_t)c];
                if (t0 < s1)
                    LTS_HIP(t.step_predict(item(-1, t0, s1, 0.5 * dtc, lts->IH, at(lts->TRH, t0, te)), s));
                if (lts->nbuf[(size_t)c])
                    LTS_HIP(dg_lts_tbuffer(fp64, lts->nbuf[(size_t)c], TB, lts->bids[(size_t)c], own_base(c),
                                           lts->TRB, tau % (int64_t(2) << c) == 0, s));
            }
            for (int c = 0; c < C; ++c) {
                const int64_t s0 = lts->start[(size_t)c], s1 = lts->start[(size_t)c + 1];
                if (s1 == s0 || (tau + 1) % (int64_t(1) << c) != 0) continue;
                if (lts->nghost[(size_t)c]) {
                    // the receiver's step is the first or the second half of
                    // a step of the next cluster up
                    const int half = ((tau + 1 - (int64_t(1) << c)) % (int64_t(2) << c)) ? 1 : 0;
                    const void *up = c + 1 < C ? own_base(c + 1) : lts->TR;
                    LTS_HIP(dg_lts_ghosts(fp64, lts->nghost[(size_t)c], TB, lts->gids[(size_t)c],
                                          lts->gkind[(size_t)c], half, up, lts->TRH, lts->TRB,
                                          at(lts->TR, lts->region[(size_t)c] + (s1 - s0), te), s));
                }
                LTS_HIP(t.step_correct(item(c, s0, s1, 0.0, lts->I, at(lts->TR, lts->region[(size_t)c], te)), s));
            }
        }
    }
#undef LTS_HIP
    return DG_OK;
}

int dg_lts_destroy(dg_lts *lts)
{
    delete lts;
    return DG_OK;
}

}  // extern "C"
