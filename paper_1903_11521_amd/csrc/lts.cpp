// Clustered local time stepping of rate 2 (the LTS of Sec. 6.4 and Table
// tab:loh1): cluster c steps with dt_c = 2^c dt0, face neighbours differ by
// at most one cluster, and the neighbour term of an element's step (Eq.
// seissol:correction_neigh) takes each neighbour's time integral over the
// element's own step interval:
//   same cluster:    the neighbour's step integral;
//   larger cluster:  the neighbour's Taylor expansion integrated over the
//                    half of its step that the element's step covers;
//   smaller cluster: the sum of the neighbour's two step integrals (a buffer
//                    filled as the neighbour steps).
// One cycle is 2^(C-1) ticks of dt0.  At each tick the clusters whose step
// starts there run their predictor; then the clusters whose step ends at
// the next tick are corrected.  Elements are numbered cluster by cluster.
//
// A cluster runs on the step kernels (predictor with time integral and face
// traces; corrector with volume, local flux and the neighbour flux of faces
// shared with its own cluster, through a cluster-relative neighbour table in
// which other clusters' elements are -1).  The faces shared with other
// clusters are added by the per-stage neighbour flux over the cluster's
// boundary range (from its first element with such a face to its end),
// reading the gathered integrals of those neighbours; the per-stage
// predictor supplies Taylor derivatives for the boundary elements that a
// smaller cluster integrates in halves.  Numbering a cluster's interior
// elements before its boundary elements keeps the boundary range short; any
// order within a cluster gives the same result.
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
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
    int PB = 0, N1 = 0;
    std::vector<int64_t> start;             // C + 1 cluster offsets
    std::vector<int64_t> bstart;            // per cluster: start of its boundary range
    std::vector<char> need_T;               // per cluster: a smaller cluster integrates it in halves
    void *T = nullptr, *I = nullptr, *Buf = nullptr, *G = nullptr, *traces = nullptr;
    int32_t *neigh_rel = nullptr;           // [E][4]: same-cluster neighbours, relative to the cluster start
    int32_t *neigh_for = nullptr;           // [E][4]: neighbours in other clusters (global ids)
    void *lists = nullptr;                  // device: gather ids, kinds and buffer ids of all clusters
    std::vector<const int32_t *> gids, bids;
    std::vector<const int8_t *> gkind;
    std::vector<int64_t> ng, nbuf;

    ~dg_lts()
    {
        for (void *p : {T, I, Buf, G, traces, (void *)neigh_rel, (void *)neigh_for, lists})
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
    const DgTable &t = plan->tab;
    if (!t.predictor || !t.neighbour_flux || !t.step_predict || !t.step_correct)
        return fail(DG_EUNSUPPORTED, "dg_lts_create: the plan's precision has no per-stage kernels");
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
    L->N1 = plan->degree + 1;
    L->start.assign((size_t)C + 1, E);
    for (int64_t e = E - 1; e >= 0; --e) L->start[(size_t)cluster[e]] = e;
    for (int c = C - 1; c >= 0; --c)
        if (L->start[(size_t)c] > L->start[(size_t)c + 1]) L->start[(size_t)c] = L->start[(size_t)c + 1];
    // host tables: per cluster its boundary range, the neighbours in other
    // clusters of its elements (each once) with their kind, and its elements
    // that have a neighbour one cluster up; the two neighbour tables
    std::vector<std::vector<int32_t>> gi((size_t)C), bi((size_t)C);
    std::vector<std::vector<int8_t>> gk((size_t)C);
    std::vector<int64_t> mark((size_t)E, -1);
    std::vector<int32_t> nrel((size_t)E * 4, -1), nfor((size_t)E * 4, -1);
    L->bstart.assign((size_t)C, 0);
    L->need_T.assign((size_t)C, 0);
    for (int c = 0; c < C; ++c) {
        const int64_t s0 = L->start[(size_t)c], s1 = L->start[(size_t)c + 1];
        int64_t first_bnd = s1;
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
                nfor[(size_t)(e * 4 + s)] = v;
                if (first_bnd == s1) first_bnd = e;
                if (dc == 1) up = true;
                if (dc == -1) L->need_T[(size_t)c] = 1;
                if (mark[(size_t)v] == c) continue;
                mark[(size_t)v] = c;
                gi[(size_t)c].push_back(v);
                gk[(size_t)c].push_back((int8_t)(dc == 1 ? 1 : 2));
            }
            if (up) bi[(size_t)c].push_back((int32_t)e);
        }
        L->bstart[(size_t)c] = first_bnd;
    }
    size_t n32 = 0, n8 = 0;
    for (int c = 0; c < C; ++c) n32 += gi[(size_t)c].size() + bi[(size_t)c].size(), n8 += gk[(size_t)c].size();
    const size_t pe = (size_t)L->PB * L->elem;
    const size_t tre = (size_t)4 * 9 * plan->Bf * L->elem;
    hipError_t h = hipSuccess;
    if (E > 0) {
        if ((h = hipMalloc(&L->T, (size_t)E * L->N1 * pe)) == hipSuccess &&
            (h = hipMalloc(&L->I, (size_t)E * pe)) == hipSuccess &&
            (h = hipMalloc(&L->Buf, (size_t)E * pe)) == hipSuccess &&
            (h = hipMalloc(&L->G, (size_t)E * pe)) == hipSuccess &&
            (h = hipMalloc(&L->traces, (size_t)E * tre)) == hipSuccess &&
            (h = hipMalloc((void **)&L->neigh_rel, (size_t)E * 16)) == hipSuccess &&
            (h = hipMalloc((void **)&L->neigh_for, (size_t)E * 16)) == hipSuccess)
            h = hipMalloc(&L->lists, n32 * 4 + n8 + 16);
        if (h == hipSuccess) h = hipMemcpy(L->neigh_rel, nrel.data(), nrel.size() * 4, hipMemcpyHostToDevice);
        if (h == hipSuccess) h = hipMemcpy(L->neigh_for, nfor.data(), nfor.size() * 4, hipMemcpyHostToDevice);
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
    L->ng.resize((size_t)C);
    L->nbuf.resize((size_t)C);
    unsigned char *dev = static_cast<unsigned char *>(L->lists);
    for (int c = 0; c < C; ++c) {
        const auto &g = gi[(size_t)c], &b = bi[(size_t)c];
        const auto &k = gk[(size_t)c];
        L->ng[(size_t)c] = (int64_t)g.size();
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
    const DgTable &t = lts->plan->tab;
    const bool fp64 = lts->elem == 8;
    const int C = lts->C, N1 = lts->N1, PB = lts->PB;
    const size_t qe = (size_t)PB * lts->elem, te = qe * N1, se = 81 * lts->elem, ae = 4 * 81;
    auto at = [](const void *p, int64_t e, size_t stride) {
        return static_cast<const char *>(p) + (size_t)e * stride;
    };
    auto atm = [](void *p, int64_t e, size_t stride) { return static_cast<char *>(p) + (size_t)e * stride; };
    const int64_t ticks = int64_t(1) << (C - 1);
    hipError_t h = hipSuccess;
#define LTS_HIP(call)                                                      \
    do {                                                                   \
        if ((h = (call)) != hipSuccess) return hip_fail(h, "dg_lts_advance"); \
    } while (0)
    const size_t tre = (size_t)4 * 9 * lts->plan->Bf * lts->elem;
    auto item = [&](int c) {
        const int64_t s0 = lts->start[(size_t)c];
        DgItem it;
        it.E = lts->start[(size_t)c + 1] - s0;
        it.dt = std::ldexp(lts->dt0, c);
        it.Q = atm(Q, s0, qe);
        it.I = atm(lts->I, s0, qe);
        it.traces = atm(lts->traces, s0, tre);
        it.star = at(star_packed, s0, se);
        it.Ap = reinterpret_cast<const double *>(at(Aplus, s0, ae * 8));
        it.Am = reinterpret_cast<const double *>(at(Aminus, s0, ae * 8));
        it.neigh = lts->neigh_rel + s0 * 4;
        it.face_rot = reinterpret_cast<const uint8_t *>(at(face_rot, s0, 4));
        it.first_block = 0;
        return it;
    };
    for (int cyc = 0; cyc < n_cycles; ++cyc) {
        for (int64_t tau = 0; tau < ticks; ++tau) {
            for (int c = 0; c < C; ++c) {
                const int64_t s0 = lts->start[(size_t)c], n = lts->start[(size_t)c + 1] - s0;
                if (n == 0 || tau % (int64_t(1) << c) != 0) continue;
                const DgItem it = item(c);
                LTS_HIP(t.step_predict(it, s));
                const int64_t b0 = lts->bstart[(size_t)c], nb = s0 + n - b0;
                if (lts->need_T[(size_t)c] && nb > 0)
                    LTS_HIP(t.predictor(nb, it.dt, at(Q, b0, qe), at(star_packed, b0, se), atm(lts->T, b0, te), s));
                if (lts->nbuf[(size_t)c])
                    LTS_HIP(dg_lts_buffer(fp64, lts->nbuf[(size_t)c], PB, lts->bids[(size_t)c], lts->I, lts->Buf,
                                          tau % (int64_t(2) << c) == 0, s));
            }
            for (int c = 0; c < C; ++c) {
                const int64_t s0 = lts->start[(size_t)c], n = lts->start[(size_t)c + 1] - s0;
                if (n == 0 || (tau + 1) % (int64_t(1) << c) != 0) continue;
                // the receiver's step inside a step of the next cluster up:
                // first half (a = 0) or second half (a = 1/2)
                const int64_t a_ticks = tau + 1 - (int64_t(1) << c);
                const double a = (a_ticks % (int64_t(2) << c)) ? 0.5 : 0.0, b = a + 0.5;
                LtsWeights w = {};
                const double dtu = std::ldexp(lts->dt0, c + 1);
                for (int d = 0; d < N1; ++d)
                    w.w[d] = dtu * (std::pow(b, d + 1) - std::pow(a, d + 1)) / (d + 1);
                LTS_HIP(dg_lts_gather(fp64, lts->ng[(size_t)c], PB, N1, lts->gids[(size_t)c], lts->gkind[(size_t)c],
                                      lts->T, lts->I, lts->Buf, lts->G, w, s));
                LTS_HIP(t.step_correct(item(c), s));
                const int64_t b0 = lts->bstart[(size_t)c], nb = s0 + n - b0;
                if (nb > 0)
                    LTS_HIP(t.neighbour_flux(nb, lts->E, lts->G, lts->neigh_for + b0 * 4,
                                             reinterpret_cast<const uint8_t *>(at(face_rot, b0, 4)),
                                             reinterpret_cast<const double *>(at(Aminus, b0, ae * 8)),
                                             atm(Q, b0, qe), s));
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
