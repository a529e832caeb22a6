// Plan object, device memory, work lists and the C ABI of esp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

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

constexpr int kMaxLds = 160 * 1024;

}  // namespace

struct esp_plan {
    int nsys = 0;
    int prec = 32;
    int device = 0;
    std::vector<esp_params> prm;
    std::vector<SysDesc> hsys;
    std::vector<Group> groups;
    Launch L{};
    std::vector<void*> allocs;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double* h_eout = nullptr;  // pinned, 4 doubles per system
    // graph replay
    bool graph_on = false;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void* g_pos = nullptr;
    const void* g_q = nullptr;
    void* g_phi = nullptr;
    void* g_F = nullptr;
    double* g_E = nullptr;

    ~esp_plan() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* p : allocs) (void)hipFree(p);
        if (h_eout) (void)hipHostFree(h_eout);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }

    template <class T>
    esp_status alloc(T** p, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess)
            return fail(ESP_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = reinterpret_cast<T*>(q);
        return ESP_OK;
    }
};

namespace {

template <class T>
std::vector<unsigned char> to_prec(const std::vector<double>& v, int prec) {
    std::vector<unsigned char> out(v.size() * (prec == 64 ? 8 : 4));
    if (prec == 64) {
        std::memcpy(out.data(), v.data(), out.size());
    } else {
        float* f = reinterpret_cast<float*>(out.data());
        for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
    }
    return out;
}

esp_status upload(esp_plan* p, void** dst, const void* src, size_t bytes) {
    unsigned char* d = nullptr;
    esp_status s = p->alloc(&d, bytes);
    if (s != ESP_OK) return s;
    HIP_TRY(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice));
    *dst = d;
    return ESP_OK;
}

// Bin edge T for a system: a divisor of n so bins tile the periodic grid
// exactly. A requested edge is rounded down to a divisor; otherwise the
// largest divisor in [8, 16] that still gives the system its share
// (`target` bins) of a few hundred spread blocks, else the smallest one.
int choose_tile(int n, int requested, long long target) {
    if (requested > 0) {
        for (int d = std::min(requested, n); d >= 4; --d)
            if (n % d == 0) return d;
        return n;
    }
    int best = 0, smallest = 0;
    for (int d = 16; d >= 8; --d) {
        if (n % d) continue;
        smallest = d;
        const long long nb = (long long)(n / d) * (n / d) * (n / d);
        if (!best && nb >= target) best = d;
    }
    if (best) return best;
    return smallest ? smallest : n;
}

esp_status build_plan(int nsys, const double* Ls, const int64_t* Ns, const double* tols, const esp_params* reqs,
                      bool per_system_req, esp_plan** out) {
    if (!out) return fail(ESP_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nsys < 1) return fail(ESP_E_INVALID, "nsys must be >= 1");
    std::unique_ptr<esp_plan> holder(new (std::nothrow) esp_plan());
    esp_plan* p = holder.get();
    if (!p) return fail(ESP_E_NOMEM, "host allocation failed");
    auto bail = [](esp_status s) { return s; };  // holder frees the plan
    HIP_TRY(hipGetDevice(&p->device));
    p->nsys = nsys;
    p->prm.resize(nsys);
    int64_t Ntot = 0;
    for (int s = 0; s < nsys; ++s) {
        const esp_params* req = reqs ? (per_system_req ? &reqs[s] : reqs) : nullptr;
        std::string msg;
        esp_status st = resolve_params(Ls[s], Ns[s], tols[s], req, &p->prm[s], msg);
        if (st != ESP_OK) return bail(fail(st, "system " + std::to_string(s) + ": " + msg));
        Ntot += Ns[s];
    }
    if (Ntot > (int64_t)1 << 30) return bail(fail(ESP_E_UNSUPPORTED, "more than 2^30 particles in one plan"));
    for (int s = 0; s < nsys; ++s) {
        const esp_params* req = reqs ? (per_system_req ? &reqs[s] : reqs) : nullptr;
        const long long target = (512LL * Ns[s] + Ntot - 1) / Ntot;
        p->prm[s].tile = choose_tile(p->prm[s].nf, req ? req->tile : 0, target);
    }
    p->prec = p->prm[0].precision;
    for (int s = 1; s < nsys; ++s)
        if (p->prm[s].precision != p->prec)
            return bail(fail(ESP_E_INVALID, "all systems of a batch must share one precision"));
    const int rb = p->prec == 64 ? 8 : 4;  // bytes per real

    // tables and descriptors
    std::vector<double> TS, Tphi, poly, tw;
    std::vector<int2> pitems, planes;
    std::vector<int4> cols;
    std::vector<std::vector<int2>> titems_by_P(13);
    p->hsys.resize(nsys);
    long long grid_off = 0, hist_total = 0, tiles_total = 0;
    int part_off = 0, tile_off = 0, nb_max = 1;
    int nmax = 0, KBmax = 1;
    for (int s = 0; s < nsys; ++s) {
        esp_params& r = p->prm[s];
        SysDesc& d = p->hsys[s];
        d.n = r.nf;
        d.P = r.P;
        d.N = (int)Ns[s];
        d.part_off = part_off;
        d.T = r.tile;
        d.tiles1 = r.nf / r.tile;
        d.E = r.tile + r.P - 1 + (r.P & 1);
        d.tile_off = tile_off;
        d.degree = r.degree;
        d.grid_off = grid_off;
        d.inv_L = 1.0 / r.L;
        d.s0 = r.s0;
        {
            // peak of the window polynomials (slightly above psi(0) at most)
            double wm = 0.0;
            std::vector<double> pc0;
            esp_params rr = r;
            window_polynomials(rr, pc0);
            for (int j = 0; j < r.P; ++j)
                for (int t = 0; t <= 64; ++t) {
                    const double y = -0.5 + t / 64.0;
                    double v = 0.0;
                    for (int m = r.degree; m >= 0; --m) v = v * y + pc0[(size_t)j * (r.degree + 1) + m];
                    wm = std::max(wm, std::fabs(v));
                }
            wm *= 1.001;
            d.wmax3 = wm * wm * wm;
        }
        std::vector<double> ts, tp, pc;
        influence_tables(r, ts, tp);
        window_polynomials(r, pc);
        d.ts_off = (int)TS.size();
        TS.insert(TS.end(), ts.begin(), ts.end());
        d.tphi_off = (int)Tphi.size();
        Tphi.insert(Tphi.end(), tp.begin(), tp.end());
        d.poly_off = (int)poly.size();
        poly.insert(poly.end(), pc.begin(), pc.end());
        d.tw_off = (int)(tw.size() / 2);
        for (int t = 0; t < r.nf; ++t) {
            const double a = 2.0 * 3.14159265358979323846 * t / r.nf;
            tw.push_back(std::cos(a));
            tw.push_back(std::sin(a));
        }
        d.pitem_off = (int)pitems.size();
        for (int c = 0; c < d.N; c += kParticleChunk) pitems.push_back(make_int2(s, c));
        d.npitem = (int)pitems.size() - d.pitem_off;
        const int nb = d.tiles1 * d.tiles1 * d.tiles1;
        d.hist_off = (int)hist_total;
        hist_total += (long long)nb * d.npitem;
        d.tb_off = tiles_total;
        tiles_total += (long long)nb * d.E * d.E * d.E;
        nb_max = std::max(nb_max, nb);
        for (int t = 0; t < nb; ++t) titems_by_P[r.P].push_back(make_int2(s, t));
        for (int x = 0; x < r.nf; ++x) planes.push_back(make_int2(s, x));
        const int hs = r.nf / 2 + 1;
        const int nch = (hs + kMaxColumns - 1) / kMaxColumns;
        const int KB = (hs + nch - 1) / nch;
        KBmax = std::max(KBmax, KB);
        d.col_off = (int)cols.size();
        for (int ky = 0; ky < r.nf; ++ky)
            for (int kz0 = 0; kz0 < hs; kz0 += KB) cols.push_back(make_int4(s, ky, kz0, std::min(KB, hs - kz0)));
        d.ncol = (int)cols.size() - d.col_off;
        nmax = std::max(nmax, r.nf);
        part_off += d.N;
        tile_off += nb;
        grid_off += (long long)r.nf * r.nf * (r.nf + 2);
    }
    // bins grouped by P
    std::vector<int2> titems;
    for (int P = 4; P <= 12; ++P) {
        if (titems_by_P[P].empty()) continue;
        Group g;
        g.P = P;
        g.off = (int)titems.size();
        g.count = (int)titems_by_P[P].size();
        int lds = 0;
        for (const int2& it : titems_by_P[P]) {
            const int E = p->hsys[it.x].E;
            lds = std::max(lds, E * E * E * 8);  // 64-bit accumulators (fixed point or double)
        }
        g.lds = lds;
        if (lds > kMaxLds) return bail(fail(ESP_E_UNSUPPORTED, "bin tile (T+P)^3 exceeds LDS; reduce tile"));
        titems.insert(titems.end(), titems_by_P[P].begin(), titems_by_P[P].end());
        p->groups.push_back(g);
    }

    Launch& L = p->L;
    L.prec = p->prec;
    L.nsys = nsys;
    L.n_pitems = (int)pitems.size();
    L.n_planes = (int)planes.size();
    L.n_cols = (int)cols.size();
    L.grid_reals = grid_off;
    L.plane_bd = nmax <= 96 ? 256 : 512;
    int need = 1;
    for (const SysDesc& d : p->hsys) need = std::max(need, ((d.n / 2 + 1) * (d.n / 2) + L.plane_bd - 1) / L.plane_bd);
    L.plane_maxit = need;
    L.plane_lds = (nmax + nmax * (nmax / 2 + 1)) * 2 * rb + (nmax + 1) * 9 * 4;  // + covering tables
    int needc = 1;
    for (const SysDesc& d : p->hsys) needc = std::max(needc, (KBmax * d.n / 2 + 255) / 256);
    L.col_maxit = needc;
    L.col_lds = (nmax + nmax * KBmax) * 2 * rb;
    if (L.plane_maxit > 12 || L.plane_lds > kMaxLds)
        return bail(fail(ESP_E_UNSUPPORTED, "grid too large for the LDS-resident plane FFT at this precision"));

    esp_status st;
    void* tmp = nullptr;
#define UP(vec, bytes) \
    if ((st = upload(p, &tmp, (vec), (bytes))) != ESP_OK) return bail(st);
    UP(p->hsys.data(), p->hsys.size() * sizeof(SysDesc));
    L.sys = reinterpret_cast<const SysDesc*>(tmp);
    UP(pitems.data(), pitems.size() * sizeof(int2));
    L.pitems = reinterpret_cast<const int2*>(tmp);
    UP(titems.data(), titems.size() * sizeof(int2));
    L.titems = reinterpret_cast<const int2*>(tmp);
    UP(planes.data(), planes.size() * sizeof(int2));
    L.planes = reinterpret_cast<const int2*>(tmp);
    UP(cols.data(), cols.size() * sizeof(int4));
    L.cols = reinterpret_cast<const int4*>(tmp);
    {
        auto b = to_prec<double>(TS, p->prec);
        UP(b.data(), b.size());
        L.TS = tmp;
    }
    {
        auto b = to_prec<double>(Tphi, p->prec);
        UP(b.data(), b.size());
        L.Tphi = tmp;
    }
    {
        auto b = to_prec<double>(poly, p->prec);
        UP(b.data(), b.size());
        L.poly = tmp;
    }
    {
        auto b = to_prec<double>(tw, p->prec);
        UP(b.data(), b.size());
        L.tw = tmp;
    }
#undef UP
    unsigned char* g = nullptr;
    if ((st = p->alloc(&g, (size_t)grid_off * rb)) != ESP_OK) return bail(st);
    L.grid = g;
    unsigned char* so = nullptr;
    if ((st = p->alloc(&so, (size_t)Ntot * 4 * rb)) != ESP_OK) return bail(st);
    L.sorted = so;
    if ((st = p->alloc(&L.perm, (size_t)Ntot)) != ESP_OK) return bail(st);
    if ((st = p->alloc(&L.rank, (size_t)Ntot)) != ESP_OK) return bail(st);
    if (hist_total > (1LL << 31) - 1) return bail(fail(ESP_E_UNSUPPORTED, "bin histogram too large"));
    if ((st = p->alloc(&L.hist, (size_t)hist_total)) != ESP_OK) return bail(st);
    L.hist_lds = nb_max * 4;
    if (L.hist_lds > kMaxLds) return bail(fail(ESP_E_UNSUPPORTED, "too many bins per system; raise tile"));
    unsigned char* tb = nullptr;
    if ((st = p->alloc(&tb, (size_t)tiles_total * rb)) != ESP_OK) return bail(st);
    L.tiles = tb;
    if ((st = p->alloc(&L.bin_start, (size_t)tile_off + 1)) != ESP_OK) return bail(st);
    if ((st = p->alloc(&L.bpart, (size_t)4 * pitems.size())) != ESP_OK) return bail(st);
    if ((st = p->alloc(&L.fx_scale, (size_t)nsys)) != ESP_OK) return bail(st);
    if ((st = p->alloc(&L.epart, cols.size())) != ESP_OK) return bail(st);
    if ((st = p->alloc(&L.eout, (size_t)4 * nsys)) != ESP_OK) return bail(st);
    HIP_TRY(hipHostMalloc((void**)&p->h_eout, sizeof(double) * 4 * nsys, hipHostMallocDefault));
    HIP_TRY(hipStreamCreate(&p->stream));
    p->own_stream = true;
    L.stream = p->stream;
    HIP_TRY(hipDeviceSynchronize());
    *out = holder.release();
    return ESP_OK;
}

// Pipeline phases (one kernel launch each, or one per window-width group).
enum Phase { kHist, kScan, kScatter, kSpread, kFftZY, kFftX, kFftYZ, kGather, kFinalize, kNumPhases };
const char* const kPhaseNames[kNumPhases] = {"hist", "scan", "scatter", "spread", "fft_zy",
                                             "fft_x_scale", "fft_yz", "gather", "finalize"};

esp_status run_phase(esp_plan* p, int ph, const void* pos, const void* q, void* phi, void* F, double* E_dev,
                     int fft_mode) {
    Launch& L = p->L;
    switch (ph) {
        case kHist:
        case kScan:
        case kScatter:
            HIP_TRY(launch_prepare(L, ph - kHist, pos, q));
            break;
        case kSpread:
            for (const Group& G : p->groups) HIP_TRY(launch_spread(L, G));
            break;
        case kFftZY:
            HIP_TRY(launch_fft(L, 0, fft_mode));
            break;
        case kFftX:
            HIP_TRY(launch_fft(L, 1, fft_mode));
            break;
        case kFftYZ:
            HIP_TRY(launch_fft(L, 2, 0));
            break;
        case kGather:
            for (const Group& G : p->groups) HIP_TRY(launch_gather(L, G, phi, F));
            break;
        case kFinalize:
            HIP_TRY(launch_finalize(L, E_dev));
            break;
    }
    return ESP_OK;
}

// Enqueue the pipeline; upto = 0 runs everything, 1..4 stop after a stage
// (diagnostics; see esp_debug_stage). With grid_in the spread is replaced by a
// copy of the caller's real grid.
esp_status enqueue(esp_plan* p, const void* pos, const void* q, void* phi, void* F, double* E_dev, int upto,
                   const void* grid_in) {
    Launch& L = p->L;
    esp_status s;
    if (grid_in) {
        HIP_TRY(hipMemcpyAsync(L.grid, grid_in, (size_t)L.grid_reals * (p->prec == 64 ? 8 : 4),
                               hipMemcpyDeviceToDevice, L.stream));
    } else {
        for (int ph = kHist; ph <= kSpread; ++ph)
            if ((s = run_phase(p, ph, pos, q, phi, F, E_dev, 0)) != ESP_OK) return s;
        if (upto == 1) {
            HIP_TRY(launch_fold(L));
            return ESP_OK;
        }
    }
    const int xmode = upto == 2 ? 1 : upto == 3 ? 2 : 0;
    if ((s = run_phase(p, kFftZY, pos, q, phi, F, E_dev, grid_in ? 3 : 0)) != ESP_OK) return s;
    if ((s = run_phase(p, kFftX, pos, q, phi, F, E_dev, xmode)) != ESP_OK) return s;
    if (upto == 2 || upto == 3) return ESP_OK;
    if ((s = run_phase(p, kFftYZ, pos, q, phi, F, E_dev, 0)) != ESP_OK) return s;
    if (upto == 4) return ESP_OK;
    for (int ph = kGather; ph <= kFinalize; ++ph)
        if ((s = run_phase(p, ph, pos, q, phi, F, E_dev, 0)) != ESP_OK) return s;
    return ESP_OK;
}

esp_status check_neutral(esp_plan* p) {
    for (int s = 0; s < p->nsys; ++s) {
        const double sq = p->h_eout[4 * s + 1], sa = p->h_eout[4 * s + 2];
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
        if (box[0] != box[1] || box[0] != box[2]) return fail(ESP_E_UNSUPPORTED, "only cubic boxes are supported");
        std::string msg;
        esp_status s = resolve_params(box[0], N, tol, req, out, msg);
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

esp_status esp_plan_create_ex(const double box[3], int64_t N, double tol, const esp_params* req, esp_plan** out) {
    try {
        if (!box) return fail(ESP_E_INVALID, "box is NULL");
        if (box[0] != box[1] || box[0] != box[2]) return fail(ESP_E_UNSUPPORTED, "only cubic boxes are supported");
        return build_plan(1, box, &N, &tol, req, false, out);
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

esp_status esp_plan_sync(esp_plan* plan) {
    if (!plan) return fail(ESP_E_INVALID, "plan is NULL");
    HIP_TRY(hipMemcpyAsync(plan->h_eout, plan->L.eout, sizeof(double) * 4 * plan->nsys, hipMemcpyDeviceToHost,
                           plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    return check_neutral(plan);
}

esp_status esp_longrange_async(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, double* E_dev) {
    if (!plan || !pos || !q) return fail(ESP_E_INVALID, "NULL argument");
    if (plan->graph_on) {
        if (!plan->gexec || pos != plan->g_pos || q != plan->g_q || phi != plan->g_phi || F != plan->g_F ||
            E_dev != plan->g_E) {
            if (plan->gexec) {
                (void)hipGraphExecDestroy(plan->gexec);
                plan->gexec = nullptr;
            }
            if (plan->graph) {
                (void)hipGraphDestroy(plan->graph);
                plan->graph = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal));
            esp_status s = enqueue(plan, pos, q, phi, F, E_dev, 0, nullptr);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(plan->stream, &g);
            if (s != ESP_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess) return fail(ESP_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            plan->graph = g;
            HIP_TRY(hipGraphInstantiate(&plan->gexec, g, nullptr, nullptr, 0));
            plan->g_pos = pos;
            plan->g_q = q;
            plan->g_phi = phi;
            plan->g_F = F;
            plan->g_E = E_dev;
        }
        HIP_TRY(hipGraphLaunch(plan->gexec, plan->stream));
        return ESP_OK;
    }
    return enqueue(plan, pos, q, phi, F, E_dev, 0, nullptr);
}

esp_status esp_longrange(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, double* E) {
    esp_status s = esp_longrange_async(plan, pos, q, phi, F, nullptr);
    if (s != ESP_OK) return s;
    if (!E) return ESP_OK;
    s = esp_plan_sync(plan);
    for (int i = 0; i < plan->nsys; ++i) E[i] = plan->h_eout[4 * i];
    return s;
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
    esp_status s = enqueue(plan, pos, q, nullptr, nullptr, nullptr, stage, grid_in);
    if (s != ESP_OK) return s;
    HIP_TRY(hipMemcpyAsync(grid_out, plan->L.grid, (size_t)plan->L.grid_reals * (plan->prec == 64 ? 8 : 4),
                           hipMemcpyDeviceToDevice, plan->stream));
    HIP_TRY(hipStreamSynchronize(plan->stream));
    return ESP_OK;
}

esp_status esp_plan_profile(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                            double* ms) {
    if (!plan || !pos || !q || !ms || reps < 1) return fail(ESP_E_INVALID, "bad argument");
    std::vector<hipEvent_t> ev(kNumPhases + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    std::vector<double> acc(kNumPhases, 0.0);
    esp_status s = ESP_OK;
    for (int r = 0; r < reps && s == ESP_OK; ++r) {
        HIP_TRY(hipEventRecord(ev[0], plan->stream));
        for (int ph = 0; ph < kNumPhases && s == ESP_OK; ++ph) {
            s = run_phase(plan, ph, pos, q, phi, F, nullptr, 0);
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

const char* esp_phase_name(int phase) { return (phase >= 0 && phase < kNumPhases) ? kPhaseNames[phase] : ""; }

void esp_plan_destroy(esp_plan* plan) { delete plan; }

}  // extern "C"
