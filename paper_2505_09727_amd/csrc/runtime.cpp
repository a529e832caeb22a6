// Plan object, device memory, work lists and the C ABI of esp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <atomic>
#include <vector>

#include "assembly.hpp"
#include "esp.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace esp;

namespace {

thread_local std::string g_err;

esp_status fail(esp_status s, const std::string& m) {
    g_err = m;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? ESP_E_NOMEM : ESP_E_DEVICE,             \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

}  // namespace

struct esp_plan {
    int nsys = 0;
    int prec = 32;
    int device = 0;
    std::vector<esp_params> prm;
    std::vector<int64_t> Ns, part_off;
    TableStore tables;
    LaunchSet ls;
    std::vector<SystemSlot> slots;
    std::vector<std::vector<double>> p3host;  // orthorhombic systems' influence tables
    unsigned char* scratch = nullptr;
    double* d_out = nullptr;   // kOutDoubles per system, contiguous
    hipStream_t stream = nullptr;  // where work is enqueued: the caller's or `own`
    hipStream_t own = nullptr;     // created by the plan when the caller gave none
    // FFT groups (grid sizes) after the first run on side streams, forked
    // from and joined back into `stream` with events, so that the groups'
    // passes overlap on the device (in a captured graph: parallel branches)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork = nullptr;
    double* h_out = nullptr;   // pinned copy of d_out
    // caller buffers the descriptors currently point to
    const void* io_pos = nullptr;
    const void* io_q = nullptr;
    void* io_phi = nullptr;
    void* io_F = nullptr;
    bool io_set = false;
    // graph replay
    bool graph_on = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double* g_E = nullptr;
    // device memory carved from the library's fixed scratch block instead of
    // allocated (esp_longrange_noalloc): nothing to free
    bool fixed_mem = false;

    ~esp_plan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamSynchronize(stream);
        if (!fixed_mem) {
            if (scratch) (void)hipFree(scratch);
            if (d_out) (void)hipFree(d_out);
        }
        if (h_out) (void)hipHostFree(h_out);
        for (hipStream_t s : side) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        for (hipEvent_t e : side_done) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (own) (void)hipStreamDestroy(own);
    }
};

namespace {

// A request with the box's y and z sides (0 where they equal the x side).
esp_params with_box(const double box[3], const esp_params* req) {
    esp_params r{};
    if (req) r = *req;
    r.Ly = box[1] == box[0] ? 0.0 : box[1];
    r.Lz = box[2] == box[0] ? 0.0 : box[2];
    return r;
}

// (Re)allocate the systems' scratch for their current tiles, carve it, and
// build the launch set. Drops a captured graph and the bound caller buffers.
esp_status assemble(esp_plan* p) {
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    if (p->graph) {
        (void)hipGraphDestroy(p->graph);
        p->graph = nullptr;
    }
    p->io_set = false;
    if (p->scratch) {
        HIP_TRY(hipStreamSynchronize(p->stream));
        HIP_TRY(hipFree(p->scratch));
        p->scratch = nullptr;
    }
    const int nsys = p->nsys;
    std::vector<size_t> off(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) off[s + 1] = off[s] + scratch_bytes(p->prm[s], p->Ns[s]);
    HIP_TRY(hipMalloc(&p->scratch, std::max<size_t>(off[nsys], 256)));
    for (int s = 0; s < nsys; ++s) {
        SystemSlot& sl = p->slots[s];
        sl.prm = p->prm[s];
        sl.N = p->Ns[s];
        std::string msg;
        esp_status st = p->tables.get(sl.prm, &sl.cls, msg);
        if (st != ESP_OK) return fail(st, msg);
        sl.scr = carve_scratch(p->scratch + off[s], sl.prm, p->Ns[s]);
        sl.scr.out = p->d_out + (size_t)kOutDoubles * s;
        if (sl.scr.p3) {
            // orthorhombic: the system's own influence table (host FP64, once)
            if (p->p3host[s].empty()) box_influence(sl.prm, *sl.cls->host, p->p3host[s]);
            const std::vector<unsigned char> b = to_prec(p->p3host[s], sl.prm.precision);
            HIP_TRY(hipMemcpy(sl.scr.p3, b.data(), b.size(), hipMemcpyHostToDevice));
        }
    }
    std::string msg;
    esp_status st = p->ls.build(p->slots, p->prec, p->stream, msg);
    if (st != ESP_OK) return fail(st, msg);
    // side streams: one per pipeline lane after the first, and one for the
    // one-block binning when the chunked binning runs beside it
    const Launch& L = p->ls.launch();
    const size_t nside = std::max<size_t>((size_t)p->ls.lanes() - 1, L.n_small > 0 && L.n_large > 0 ? 1 : 0);
    if (nside && !p->fork) HIP_TRY(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    while (p->side.size() < nside) {
        hipStream_t s = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        p->side.push_back(s);
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->side_done.push_back(e);
    }
    HIP_TRY(hipStreamSynchronize(p->stream));
    return ESP_OK;
}

esp_status build_plan(int nsys, const double* Ls, const int64_t* Ns, const double* tols, const esp_params* reqs,
                      bool per_system_req, esp_plan** out) {
    if (!out) return fail(ESP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nsys < 1) return fail(ESP_E_INVALID, "nsys must be >= 1");
    std::unique_ptr<esp_plan> holder(new (std::nothrow) esp_plan());
    esp_plan* p = holder.get();
    if (!p) return fail(ESP_E_NOMEM, "host allocation failed");
    HIP_TRY(hipGetDevice(&p->device));
    p->nsys = nsys;
    p->prm.resize(nsys);
    p->Ns.assign(Ns, Ns + nsys);
    int64_t Ntot = 0;
    for (int s = 0; s < nsys; ++s) {
        const esp_params* req = reqs ? (per_system_req ? &reqs[s] : reqs) : nullptr;
        std::string msg;
        esp_status st = resolve_params(Ls[s], Ns[s], tols[s], req, &p->prm[s], msg);
        if (st != ESP_OK) return fail(st, "system " + std::to_string(s) + ": " + msg);
        p->part_off.push_back(Ntot);
        Ntot += Ns[s];
    }
    if (Ntot > (int64_t)1 << 31) return fail(ESP_E_UNSUPPORTED, "more than 2^31 particles in one plan");
    for (int s = 0; s < nsys; ++s) {
        const esp_params* req = reqs ? (per_system_req ? &reqs[s] : reqs) : nullptr;
        // each system's share of a few hundred spread blocks
        const long long target = (512LL * Ns[s] + Ntot - 1) / Ntot;
        p->prm[s].tile = choose_tile(p->prm[s].nf, req ? req->tile : 0, target);
    }
    p->prec = p->prm[0].precision;
    for (int s = 1; s < nsys; ++s)
        if (p->prm[s].precision != p->prec) return fail(ESP_E_INVALID, "all systems of a batch must share one precision");

    HIP_TRY(hipMalloc(&p->d_out, sizeof(double) * kOutDoubles * nsys));
    HIP_TRY(hipMemset(p->d_out, 0, sizeof(double) * kOutDoubles * nsys));
    HIP_TRY(hipHostMalloc((void**)&p->h_out, sizeof(double) * kOutDoubles * nsys, hipHostMallocDefault));
    if (reqs && reqs[0].stream) {
        p->stream = static_cast<hipStream_t>(reqs[0].stream);  // the caller's
    } else {
        HIP_TRY(hipStreamCreate(&p->own));
        p->stream = p->own;
    }
    for (int s = 0; s < nsys; ++s) p->prm[s].stream = p->stream;
    p->slots.resize(nsys);
    p->p3host.resize(nsys);
    esp_status st = assemble(p);
    if (st != ESP_OK) return st;
    *out = holder.release();
    return ESP_OK;
}

// Point the descriptors at the caller's concatenated arrays (uploaded only
// when the pointers change).
esp_status bind_io(esp_plan* p, const void* pos, const void* q, void* phi, void* F) {
    if (p->io_set && pos == p->io_pos && q == p->io_q && phi == p->io_phi && F == p->io_F) return ESP_OK;
    const size_t rb = p->prec == 64 ? 8 : 4;
    for (int s = 0; s < p->nsys; ++s) {
        const size_t o = (size_t)p->part_off[s];
        p->ls.set_io(s, static_cast<const unsigned char*>(pos) + 3 * o * rb,
                     static_cast<const unsigned char*>(q) + o * rb,
                     phi ? static_cast<unsigned char*>(phi) + o * rb : nullptr,
                     F ? static_cast<unsigned char*>(F) + 3 * o * rb : nullptr);
    }
    std::string msg;
    esp_status st = p->ls.upload_descriptors(msg);
    if (st != ESP_OK) return fail(st, msg);
    p->io_pos = pos;
    p->io_q = q;
    p->io_phi = phi;
    p->io_F = F;
    p->io_set = true;
    return ESP_OK;
}

// Pipeline phases (one kernel launch each, or one per window-width group).
enum Phase { kHist, kScan, kScatter, kLocal, kSpread, kFftZY, kFftX, kFftYZ, kGather, kFinalize, kNumPhases };
static_assert(kNumPhases == ESP_NUM_PHASES, "esp.h's phase count must match the pipeline");
const char* const kPhaseNames[kNumPhases] = {"hist", "scan", "scatter", "local", "spread", "fft_zy",
                                             "fft_x_scale", "fft_yz", "gather", "finalize"};

esp_status run_phase(esp_plan* p, int ph, double* E_dev, int fft_mode) {
    const Launch& L = p->ls.launch();
    switch (ph) {
        case kHist:
        case kScan:
        case kScatter:
            HIP_TRY(launch_prepare(L, ph - kHist));
            break;
        case kLocal:
            HIP_TRY(launch_local(L));
            break;
        case kSpread:
            for (const Group& G : p->ls.groups()) HIP_TRY(launch_spread(L, G));
            break;
        case kFftZY:
            for (const FftGroup& G : p->ls.fft_groups()) HIP_TRY(launch_fft(L, G, 0, fft_mode));
            break;
        case kFftX:
            for (const FftGroup& G : p->ls.fft_groups()) HIP_TRY(launch_fft(L, G, 1, fft_mode));
            break;
        case kFftYZ:
            for (const FftGroup& G : p->ls.fft_groups()) HIP_TRY(launch_fft(L, G, 2, 0, E_dev));
            break;
        case kGather:
            for (const Group& G : p->ls.groups()) HIP_TRY(launch_gather(L, G));
            break;
        case kFinalize:
            HIP_TRY(launch_finalize(L, E_dev));
            break;
    }
    return ESP_OK;
}

// Enqueue the pipeline; upto = 0 runs everything, 1..4 stop after a stage
// (diagnostics; see esp_debug_stage). With grid_in, system 0's spread is
// replaced by a copy of the caller's real grid.
esp_status enqueue(esp_plan* p, double* E_dev, int upto, const void* grid_in) {
    esp_status s;
    if (grid_in) {
        const esp_params& r = p->prm[0];
        HIP_TRY(hipMemcpyAsync(p->slots[0].scr.grid, grid_in,
                               (size_t)r.nf * r.nf * (r.nf + 2) * (p->prec == 64 ? 8 : 4), hipMemcpyDeviceToDevice,
                               p->stream));
    } else {
        const Launch& L = p->ls.launch();
        int ph = kHist;
        if (L.n_small > 0 && L.n_large > 0 && !p->side.empty()) {
            // the one-block binning of the small systems on a side stream,
            // beside the chunked binning of the others
            HIP_TRY(hipEventRecord(p->fork, p->stream));
            HIP_TRY(hipStreamWaitEvent(p->side[0], p->fork, 0));
            Launch Ls = L;
            Ls.stream = p->side[0];
            HIP_TRY(launch_bin_small(Ls));
            HIP_TRY(hipEventRecord(p->side_done[0], p->side[0]));
            for (int q = 0; q < 3; ++q) HIP_TRY(launch_prepare(L, q, false));
            HIP_TRY(hipStreamWaitEvent(p->stream, p->side_done[0], 0));
            ph = kLocal;
        }
        const int lanes = p->ls.lanes();
        if (upto == 0 && lanes > 1 && (int)p->side.size() >= lanes - 1) {
            // the pipeline lanes: each runs its systems' spread, FFT passes
            // and gather on its own stream (lane 0 the plan's, lane l side
            // stream l - 1), forked after the binning and joined before the
            // finalisation; launches go in phase order across the lanes
            for (; ph <= kLocal; ++ph)
                if ((s = run_phase(p, ph, E_dev, 0)) != ESP_OK) return s;
            HIP_TRY(hipEventRecord(p->fork, p->stream));
            for (int l = 1; l < lanes; ++l) HIP_TRY(hipStreamWaitEvent(p->side[l - 1], p->fork, 0));
            std::vector<Launch> Ll(lanes, L);
            for (int l = 1; l < lanes; ++l) Ll[l].stream = p->side[l - 1];
            for (const Group& G : p->ls.groups()) HIP_TRY(launch_spread(Ll[G.lane], G));
            const std::vector<FftGroup>& fg = p->ls.fft_groups();
            for (int pass = 0; pass < 3; ++pass)
                for (const FftGroup& G : fg) HIP_TRY(launch_fft(Ll[G.lane], G, pass, 0, pass == 2 ? E_dev : nullptr));
            for (const Group& G : p->ls.groups()) HIP_TRY(launch_gather(Ll[G.lane], G));
            for (int l = 1; l < lanes; ++l) {
                HIP_TRY(hipEventRecord(p->side_done[l - 1], p->side[l - 1]));
                HIP_TRY(hipStreamWaitEvent(p->stream, p->side_done[l - 1], 0));
            }
            return run_phase(p, kFinalize, E_dev, 0);
        }
        for (; ph <= kSpread; ++ph)
            if ((s = run_phase(p, ph, E_dev, 0)) != ESP_OK) return s;
        if (upto == 1) {
            HIP_TRY(launch_fold(p->ls.launch()));
            return ESP_OK;
        }
    }
    const int xmode = upto == 2 ? 1 : upto == 3 ? 2 : 0;
    if ((s = run_phase(p, kFftZY, E_dev, (grid_in ? 3 : 0) | (xmode << 2))) != ESP_OK) return s;
    if ((s = run_phase(p, kFftX, E_dev, xmode)) != ESP_OK) return s;
    if (upto == 2 || upto == 3) return ESP_OK;
    if ((s = run_phase(p, kFftYZ, E_dev, 0)) != ESP_OK) return s;
    if (upto == 4) return ESP_OK;
    for (int ph = kGather; ph <= kFinalize; ++ph)
        if ((s = run_phase(p, ph, E_dev, 0)) != ESP_OK) return s;
    return ESP_OK;
}

esp_status check_neutral(esp_plan* p) {
    for (int s = 0; s < p->nsys; ++s) {
        const double sq = p->h_out[kOutDoubles * s + 1], sa = p->h_out[kOutDoubles * s + 2];
        if (std::fabs(sq) > 1e-6 * sa)
            return fail(ESP_E_NOT_NEUTRAL, "system " + std::to_string(s) + " is not charge neutral (sum q = " +
                                               std::to_string(sq) + ")");
    }
    return ESP_OK;
}

}  // namespace

extern "C" {

const char* esp_last_error(void) { return g_err.c_str(); }

const char* esp_version(void) { return "esp-mi355x 0.1 (gfx950)"; }

esp_status esp_plan_query(const double box[3], int64_t N, double tol, const esp_params* req, esp_params* out) {
    try {
        if (!box || !out) return fail(ESP_E_INVALID, "NULL argument");
        const esp_params rq = with_box(box, req);
        std::string msg;
        esp_status s = resolve_params(box[0], N, tol, &rq, out, msg);
        if (s != ESP_OK) return fail(s, msg);
        return ESP_OK;
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}

esp_status esp_window_coeffs(const esp_params* resolved, double* coef) {
    if (!resolved || !coef) return fail(ESP_E_INVALID, "NULL argument");
    esp_params r = *resolved;
    std::vector<double> c;
    window_polynomials(r, c);
    std::memcpy(coef, c.data(), c.size() * sizeof(double));
    return ESP_OK;
}

esp_status esp_local_coeffs(const esp_params* resolved, double* A, double* B, int* pieces, int* degree) {
    if (!resolved || !A || !B || !pieces || !degree) return fail(ESP_E_INVALID, "NULL argument");
    if (!(resolved->h > 0) || !(resolved->rc > 0) || !(resolved->c > 0))
        return fail(ESP_E_INVALID, "parameters are not resolved (use esp_plan_query)");
    try {
        std::vector<double> a, b;
        int d = 0;
        local_polynomials(resolved->method, resolved->c, grid_rho(*resolved), d, a, b);
        std::memcpy(A, a.data(), a.size() * sizeof(double));
        std::memcpy(B, b.data(), b.size() * sizeof(double));
        *pieces = kLocalPieces;
        *degree = d;
        return ESP_OK;
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}

esp_status esp_influence_tables(const esp_params* resolved, double* TS, double* Tphi) {
    if (!resolved || !TS || !Tphi) return fail(ESP_E_INVALID, "NULL argument");
    std::vector<double> a, b;
    influence_tables(*resolved, a, b);
    std::memcpy(TS, a.data(), a.size() * sizeof(double));
    std::memcpy(Tphi, b.data(), b.size() * sizeof(double));
    return ESP_OK;
}

esp_status esp_local_kernel(const esp_params* resolved, const double* r, int64_t n, double* Lr, double* dLr) {
    if (!resolved || (!r && n) || !Lr || !dLr) return fail(ESP_E_INVALID, "NULL argument");
    for (int64_t i = 0; i < n; ++i)
        if (!(r[i] > 0)) return fail(ESP_E_INVALID, "radii must be positive");
    local_kernel(*resolved, r, n, Lr, dLr);
    return ESP_OK;
}

esp_status esp_warm_tables(const double* tols, int ntol, int nf_max, int threads) {
    try {
        if (!tols || ntol < 1) return fail(ESP_E_INVALID, "no tolerances");
        if (nf_max <= 0 || nf_max > 144) nf_max = 144;
        std::vector<std::pair<int, double>> work;
        for (int i = 0; i < ntol; ++i) {
            const int P = order_for_tol(tols[i]);
            if (!(tols[i] > 0) || P > 12) return fail(ESP_E_UNSUPPORTED, "tolerance outside the supported orders");
            for (int n = std::max(8, P); n <= nf_max; ++n)  // grids narrower than the window never occur
                if (is_smooth(n)) work.emplace_back(n, tols[i]);
        }
        if (threads <= 0) threads = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
        std::atomic<size_t> next{0};
        std::atomic<int> bad{0};
        auto worker = [&] {
            for (size_t k; (k = next++) < work.size();) {
                esp_params req{}, r{};
                req.nf = work[k].first;
                std::string msg;
                // any box with this grid: the class does not depend on L
                if (resolve_params(1.25 * req.nf, 1000, work[k].second, &req, &r, msg) != ESP_OK) {
                    ++bad;
                    continue;
                }
                (void)class_tables(r);
            }
        };
        std::vector<std::thread> pool;
        for (int t = 0; t < threads; ++t) pool.emplace_back(worker);
        for (auto& t : pool) t.join();
        return bad ? fail(ESP_E_INVALID, "some tolerances could not be resolved") : ESP_OK;
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}

esp_status esp_plan_create_ex(const double box[3], int64_t N, double tol, const esp_params* req, esp_plan** out) {
    try {
        if (!box) return fail(ESP_E_INVALID, "box is NULL");
        const esp_params rq = with_box(box, req);
        return build_plan(1, box, &N, &tol, &rq, false, out);
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}

esp_status esp_plan_create(const double box[3], int64_t N, double tol, esp_plan** out) {
    return esp_plan_create_ex(box, N, tol, nullptr, out);
}

esp_status esp_batch_create(int nsys, const double* L, const int64_t* N, const double* tol, const esp_params* reqs,
                            esp_plan** out) {
    try {
        if (!L || !N || !tol) return fail(ESP_E_INVALID, "NULL argument");
        return build_plan(nsys, L, N, tol, reqs, true, out);
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}

esp_status esp_plan_get_params(const esp_plan* plan, int sys, esp_params* out) {
    if (!plan || !out) return fail(ESP_E_INVALID, "NULL argument");
    if (sys < 0 || sys >= plan->nsys) return fail(ESP_E_INVALID, "system index out of range");
    *out = plan->prm[sys];
    return ESP_OK;
}

int esp_plan_num_systems(const esp_plan* plan) { return plan ? plan->nsys : 0; }

void* esp_plan_stream(const esp_plan* plan) { return plan ? (void*)plan->stream : nullptr; }

esp_status esp_plan_set_stream(esp_plan* plan, void* stream) {
    if (!plan) return fail(ESP_E_INVALID, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s == plan->stream) return ESP_OK;
    // the scratch must not be in use on two streams at once
    HIP_TRY(hipStreamSynchronize(plan->stream));
    plan->stream = s;
    plan->ls.set_stream(s);
    for (auto& r : plan->prm) r.stream = stream;
    for (auto& sl : plan->slots) sl.prm.stream = stream;
    return ESP_OK;
}

esp_status esp_plan_shortrange_coeffs(const esp_plan* plan, double* coef, int* npieces, int* degree) {
    if (!plan || !coef || !npieces || !degree) return fail(ESP_E_INVALID, "NULL argument");
    double A[ESP_LOCAL_COEF_MAX], B[ESP_LOCAL_COEF_MAX];
    const esp_status s = esp_local_coeffs(&plan->prm[0], A, B, npieces, degree);
    if (s != ESP_OK) return s;
    const int m = *npieces * (*degree + 1);  // A, then B right after it
    std::memcpy(coef, A, sizeof(double) * m);
    std::memcpy(coef + m, B, sizeof(double) * m);
    return ESP_OK;
}

esp_status esp_plan_sync(esp_plan* plan) {
    if (!plan) return fail(ESP_E_INVALID, "plan is NULL");
    HIP_TRY(hipMemcpyAsync(plan->h_out, plan->d_out, sizeof(double) * kOutDoubles * plan->nsys, hipMemcpyDeviceToHost,
                           plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    return check_neutral(plan);
}

esp_status esp_longrange_async(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, double* E_dev) {
    if (!plan || !pos || !q) return fail(ESP_E_INVALID, "NULL argument");
    const bool moved = !plan->io_set || pos != plan->io_pos || q != plan->io_q || phi != plan->io_phi ||
                       F != plan->io_F;
    esp_status s = bind_io(plan, pos, q, phi, F);
    if (s != ESP_OK) return s;
    if (plan->graph_on) {
        if (!plan->gexec || moved || E_dev != plan->g_E) {
            if (plan->gexec) {
                (void)hipGraphExecDestroy(plan->gexec);
                plan->gexec = nullptr;
            }
            if (plan->graph) {
                (void)hipGraphDestroy(plan->graph);
                plan->graph = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal));
            s = enqueue(plan, E_dev, 0, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(plan->stream, &g);
            if (s != ESP_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess) return fail(ESP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            plan->graph = g;
            HIP_TRY(hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
            plan->g_E = E_dev;
        }
        HIP_TRY(hipGraphLaunch(plan->gexec, plan->stream));
        return ESP_OK;
    }
    return enqueue(plan, E_dev, 0, nullptr);
}

esp_status esp_longrange(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, double* E) {
    esp_status s = esp_longrange_async(plan, pos, q, phi, F, nullptr);
    if (s != ESP_OK) return s;
    if (!E) return ESP_OK;
    s = esp_plan_sync(plan);
    for (int i = 0; i < plan->nsys; ++i) E[i] = plan->h_out[kOutDoubles * i];
    return s;
}

esp_status esp_batch_longrange(esp_plan* batch, const void* pos, const void* q, void* phi, void* F, double* E) {
    return esp_longrange(batch, pos, q, phi, F, E);
}

// Sweeps over the autotuner's candidates; each keeps its fastest.
constexpr int kTuneRounds = 3;

esp_status esp_plan_autotune(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                             int* tiles_out) {
    if (!plan || !pos || !q || reps < 1) return fail(ESP_E_INVALID, "bad argument");
    // groups of systems sharing (grid, window width), largest work first
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int s = 0; s < plan->nsys; ++s) groups[{plan->prm[s].nf, plan->prm[s].P}].push_back(s);
    std::vector<std::pair<double, std::vector<int>>> order;
    for (auto& kv : groups) {
        double w = 0.0;
        for (int s : kv.second) w += (double)plan->Ns[s];
        order.push_back({w, kv.second});
    }
    std::sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto time_steps = [&](double* ms) -> esp_status {
        esp_status st = bind_io(plan, pos, q, phi, F);
        if (st != ESP_OK) return st;
        if ((st = enqueue(plan, nullptr, 0, nullptr)) != ESP_OK) return st;  // warm-up
        HIP_TRY(hipEventRecord(e0, plan->stream));
        for (int r = 0; r < reps; ++r)
            if ((st = enqueue(plan, nullptr, 0, nullptr)) != ESP_OK) return st;
        HIP_TRY(hipEventRecord(e1, plan->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e0, e1));
        *ms = t;
        return ESP_OK;
    };
    esp_status st = ESP_OK;
    for (auto& g : order) {
        const std::vector<int>& sys = g.second;
        const esp_params& r0 = plan->prm[sys[0]];
        const int tile0 = r0.tile, path0 = r0.fft_passes;  // the plan's current choice
        const std::vector<int> cand = tile_candidates(r0.nf, r0.P);
        const int npaths = fft_fused_lds(r0.nf, plan->prec) <= kMaxLds ? 2 : 1;
        if (cand.size() * npaths < 2) continue;
        // each candidate's time is its best over kTuneRounds interleaved
        // sweeps: steps of a plan with concurrent lanes vary by a few
        // percent from one replay to the next, enough for a single sweep
        // to keep a slower choice
        std::vector<std::pair<int, int>> cands;  // (path, T)
        for (int path = 0; path < npaths; ++path)
            for (int T : cand) cands.push_back({path, T});
        std::vector<double> best_of(cands.size(), 1e30);
        for (int round = 0; round < kTuneRounds && st == ESP_OK; ++round)
            for (size_t k = 0; k < cands.size(); ++k) {
                for (int s : sys) {
                    plan->prm[s].tile = cands[k].second;
                    plan->prm[s].fft_passes = cands[k].first;
                }
                if ((st = assemble(plan)) != ESP_OK) break;
                double ms = 0.0;
                if ((st = time_steps(&ms)) != ESP_OK) break;
                best_of[k] = std::min(best_of[k], ms);
            }
        if (st != ESP_OK) break;
        // the plan's current choice stays unless another is 2% faster
        size_t kb = (size_t)(std::min_element(best_of.begin(), best_of.end()) - best_of.begin());
        for (size_t k = 0; k < cands.size(); ++k)
            if (cands[k].second == tile0 && cands[k].first == path0 && best_of[kb] > 0.98 * best_of[k]) kb = k;
        const int best = cands[kb].second, best_path = cands[kb].first;
        for (int s : sys) {
            plan->prm[s].tile = best;
            plan->prm[s].fft_passes = best_path;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ESP_OK) return st;
    if ((st = assemble(plan)) != ESP_OK) return st;
    if (tiles_out)
        for (int s = 0; s < plan->nsys; ++s) tiles_out[s] = plan->prm[s].tile;
    return ESP_OK;
}

esp_status esp_plan_set_graph(esp_plan* plan, int enable) {
    if (!plan) return fail(ESP_E_INVALID, "plan is NULL");
    plan->graph_on = enable != 0;
    return ESP_OK;
}

esp_status esp_debug_stage(esp_plan* plan, const void* pos, const void* q, const void* grid_in, int stage,
                           void* grid_out) {
    if (!plan || !grid_out) return fail(ESP_E_INVALID, "NULL argument");
    if (stage < 1 || stage > 4) return fail(ESP_E_INVALID, "stage must be 1..4");
    if (!grid_in && (!pos || !q)) return fail(ESP_E_INVALID, "pos and q are required without grid_in");
    if (grid_in && stage == 1) return fail(ESP_E_INVALID, "stage 1 needs particles");
    esp_status s;
    if (!grid_in && (s = bind_io(plan, pos, q, nullptr, nullptr)) != ESP_OK) return s;
    if ((s = enqueue(plan, nullptr, stage, grid_in)) != ESP_OK) return s;
    const esp_params& r = plan->prm[0];
    HIP_TRY(hipMemcpyAsync(grid_out, plan->slots[0].scr.grid, (size_t)r.nf * r.nf * (r.nf + 2) * (plan->prec == 64 ? 8 : 4),
                           hipMemcpyDeviceToDevice, plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    return ESP_OK;
}

esp_status esp_debug_gather(esp_plan* plan, const void* pos, const void* q, const void* grid_c, void* phi,
                            void* F) {
    if (!plan || !pos || !q || !grid_c) return fail(ESP_E_INVALID, "NULL argument");
    const esp_params& r = plan->prm[0];
    if (plan->nsys != 1 || r.local || r.force_method != 0)
        return fail(ESP_E_UNSUPPORTED, "the gather stage alone needs a single-system long-range plan with AD forces");
    esp_status s = bind_io(plan, pos, q, phi, F);
    if (s != ESP_OK) return s;
    for (int ph = kHist; ph <= kScatter; ++ph)
        if ((s = run_phase(plan, ph, nullptr, 0)) != ESP_OK) return s;
    HIP_TRY(hipMemcpyAsync(plan->slots[0].scr.grid, grid_c,
                           (size_t)r.nf * r.nf * (r.nf + 2) * (plan->prec == 64 ? 8 : 4), hipMemcpyDeviceToDevice,
                           plan->stream));
    if ((s = run_phase(plan, kGather, nullptr, 0)) != ESP_OK) return s;
    HIP_TRY(hipStreamSynchronize(plan->stream));
    return ESP_OK;
}

esp_status esp_plan_profile(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                            double* ms) {
    if (!plan || !pos || !q || !ms || reps < 1) return fail(ESP_E_INVALID, "bad argument");
    esp_status s = bind_io(plan, pos, q, phi, F);
    if (s != ESP_OK) return s;
    std::vector<hipEvent_t> ev(kNumPhases + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    std::vector<double> acc(kNumPhases, 0.0);
    for (int r = 0; r < reps && s == ESP_OK; ++r) {
        // an untimed pass first keeps the GPU busy while the timed pass is
        // enqueued, so no phase is charged for host launch latency
        for (int ph = 0; ph < kNumPhases && s == ESP_OK; ++ph) s = run_phase(plan, ph, nullptr, 0);
        HIP_TRY(hipEventRecord(ev[0], plan->stream));
        for (int ph = 0; ph < kNumPhases && s == ESP_OK; ++ph) {
            s = run_phase(plan, ph, nullptr, 0);
            HIP_TRY(hipEventRecord(ev[ph + 1], plan->stream));
        }
        HIP_TRY(hipEventSynchronize(ev[kNumPhases]));
        for (int ph = 0; ph < kNumPhases; ++ph) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, ev[ph], ev[ph + 1]));
            acc[ph] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int ph = 0; ph < kNumPhases; ++ph) ms[ph] = acc[ph] / reps;
    return s;
}

esp_status esp_plan_profile_launches(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                                     int phase, int max, double* ms, int64_t* particles, int64_t* points,
                                     int64_t* blocks, int* count) {
    if (!plan || !pos || !q || !ms || !particles || !points || !blocks || !count || reps < 1 || max < 0)
        return fail(ESP_E_INVALID, "bad argument");
    if (phase != kSpread && phase != kGather) return fail(ESP_E_INVALID, "phase must be spread or gather");
    esp_status s = bind_io(plan, pos, q, phi, F);
    if (s != ESP_OK) return s;
    const std::vector<Group>& gs = plan->ls.groups();
    const int ng = (int)gs.size();
    *count = std::min(ng, max);
    // particles and grid points of each launch: its systems' sums
    for (int k = 0; k < *count; ++k) {
        particles[k] = 0;
        points[k] = 0;
        blocks[k] = gs[k].count;  // the launch's grid (XCD-ordered list, padding included)
    }
    for (int s2 = 0; s2 < plan->nsys; ++s2) {
        const SysDesc& d = plan->ls.desc(s2);
        for (int k = 0; k < *count; ++k)
            if (gs[k].P == d.P && gs[k].lane == plan->ls.lane_of(s2)) {
                particles[k] += d.N;
                points[k] += (int64_t)d.n * d.n * d.n;
            }
    }
    const Launch& L = plan->ls.launch();
    std::vector<hipEvent_t> ev(ng + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    std::vector<double> acc(ng, 0.0);
    for (int r = 0; r < reps && s == ESP_OK; ++r) {
        for (int ph = 0; ph < kNumPhases && s == ESP_OK; ++ph) s = run_phase(plan, ph, nullptr, 0);
        for (int ph = 0; ph < phase && s == ESP_OK; ++ph) s = run_phase(plan, ph, nullptr, 0);
        HIP_TRY(hipEventRecord(ev[0], plan->stream));
        for (int k = 0; k < ng; ++k) {
            HIP_TRY(phase == kSpread ? launch_spread(L, gs[k]) : launch_gather(L, gs[k]));
            HIP_TRY(hipEventRecord(ev[k + 1], plan->stream));
        }
        for (int ph = phase + 1; ph < kNumPhases && s == ESP_OK; ++ph) s = run_phase(plan, ph, nullptr, 0);
        HIP_TRY(hipEventSynchronize(ev[ng]));
        for (int k = 0; k < ng; ++k) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
            acc[k] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k < *count; ++k) ms[k] = acc[k] / reps;
    return s;
}

int esp_num_phases(void) { return kNumPhases; }

const char* esp_phase_name(int phase) { return (phase >= 0 && phase < kNumPhases) ? kPhaseNames[phase] : ""; }

void esp_plan_destroy(esp_plan* plan) { delete plan; }

}  // extern "C"

// ---------------------------------------------------------------------------
// One long-range evaluation without allocating device memory. Every buffer
// of the pipeline (sorted particles, bins, grids, tiles, tables, launch
// lists, partial sums, the per-system results) is carved from `scratch`, a
// fixed block in device memory that each GPU holds for the life of the
// process. Host code reaches it only through the device address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in); that address is looked up once per device, on the
// first call there.
namespace {

static __device__ __align__(256) unsigned char scratch[ESP_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;  // device ordinal -> address of its scratch

esp_status scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(ESP_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch block");
        it = g_scratch_ptr.emplace(dev, static_cast<unsigned char*>(ptr)).first;
    }
    *out = it->second;
    return ESP_OK;
}

}  // namespace

extern "C" esp_status esp_longrange_noalloc(const double box[3], int64_t N, double tol, const esp_params* req,
                                            const void* pos, const void* q, void* phi, void* F, double* E,
                                            void* stream) {
    try {
        if (!box || !pos || !q) return fail(ESP_E_INVALID, "NULL argument");
        esp_params rq = with_box(box, req);
        std::unique_ptr<esp_plan> holder(new (std::nothrow) esp_plan());
        esp_plan* p = holder.get();
        if (!p) return fail(ESP_E_NOMEM, "host allocation failed");
        p->fixed_mem = true;
        HIP_TRY(hipGetDevice(&p->device));
        p->nsys = 1;
        p->prm.resize(1);
        p->Ns.assign(1, N);
        p->part_off.assign(1, 0);
        std::string msg;
        esp_status st = resolve_params(box[0], N, tol, &rq, &p->prm[0], msg);
        if (st != ESP_OK) return fail(st, msg);
        esp_params& r = p->prm[0];
        r.tile = choose_tile(r.nf, req ? req->tile : 0, 512);
        p->prec = r.precision;
        p->stream = static_cast<hipStream_t>(stream);
        r.stream = stream;
        unsigned char* base = nullptr;
        if ((st = scratch_of_current_device(&base)) != ESP_OK) return st;
        FixedBlock arena{base, (size_t)ESP_NOALLOC_SCRATCH_BYTES, 0};
        const size_t need = scratch_bytes(r, N);
        p->d_out = static_cast<double*>(arena.take(sizeof(double) * kOutDoubles));
        p->scratch = static_cast<unsigned char*>(arena.take(need));
        if (!p->d_out || !p->scratch)
            return fail(ESP_E_UNSUPPORTED, "this system needs " + std::to_string(need) +
                                               " bytes of scratch; the no-allocation entry point holds " +
                                               std::to_string((size_t)ESP_NOALLOC_SCRATCH_BYTES));
        p->tables.set_arena(&arena);
        p->ls.set_arena(&arena);
        p->slots.resize(1);
        p->p3host.resize(1);
        SystemSlot& sl = p->slots[0];
        sl.prm = r;
        sl.N = N;
        if ((st = p->tables.get(sl.prm, &sl.cls, msg)) != ESP_OK) return fail(st, msg);
        sl.scr = carve_scratch(p->scratch, sl.prm, N);
        sl.scr.out = p->d_out;
        if (sl.scr.p3) {
            box_influence(sl.prm, *sl.cls->host, p->p3host[0]);
            const std::vector<unsigned char> b = to_prec(p->p3host[0], sl.prm.precision);
            HIP_TRY(hipMemcpy(sl.scr.p3, b.data(), b.size(), hipMemcpyHostToDevice));
        }
        if ((st = p->ls.build(p->slots, p->prec, p->stream, msg)) != ESP_OK) return fail(st, msg);
        if ((st = bind_io(p, pos, q, phi, F)) != ESP_OK) return st;
        if ((st = enqueue(p, nullptr, 0, nullptr)) != ESP_OK) return st;
        double out[kOutDoubles];
        HIP_TRY(hipMemcpyAsync(out, p->d_out, sizeof(out), hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipStreamSynchronize(p->stream));
        if (E) *E = out[0];
        if (std::fabs(out[1]) > 1e-6 * out[2])
            return fail(ESP_E_NOT_NEUTRAL, "the system is not charge neutral (sum q = " + std::to_string(out[1]) + ")");
        return ESP_OK;
    } catch (const std::exception& e) {
        return fail(ESP_E_INVALID, e.what());
    }
}
