// Launch-set assembly (see assembly.hpp).
#include "assembly.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>

namespace esp {

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

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int nbins(const esp_params& p) {
    const int t1 = p.nf / p.tile;
    return t1 * t1 * t1;
}

int tile_edge(const esp_params& p) { return p.tile + p.P - 1 + (p.P & 1); }

int npitems(int64_t N) { return (int)((N + kParticleChunk - 1) / kParticleChunk); }

}  // namespace

TableStore::~TableStore() {
    for (void* p : allocs_) (void)hipFree(p);
}

esp_status TableStore::get(const esp_params& p, const DeviceClass** out, std::string& msg) {
    std::shared_ptr<const ClassTables> t = class_tables(p);
    const auto key = std::make_pair(t.get(), p.precision);
    auto it = dev_.find(key);
    if (it != dev_.end()) {
        *out = &it->second;
        return ESP_OK;
    }
    DeviceClass d;
    d.host = t.get();
    // local-part polynomials zero-padded to kLocalMaxDegree: A then B
    std::vector<double> lcoef(2 * (kLocalMaxDegree + 1), 0.0);
    std::copy(t->lA.begin(), t->lA.end(), lcoef.begin());
    std::copy(t->lB.begin(), t->lB.end(), lcoef.begin() + kLocalMaxDegree + 1);
    const std::vector<double>* src[5] = {&t->TS, &t->Tphi, &t->poly, &t->tw, &lcoef};
    void** dst[5] = {&d.TS, &d.Tphi, &d.poly, &d.tw, &d.lcoef};
    for (int i = 0; i < 5; ++i) {
        auto b = to_prec(*src[i], p.precision);
        void* q = nullptr;
        if (arena_) {
            q = arena_->take(std::max<size_t>(b.size(), 16));
            if (!q) {
                msg = "the fixed scratch block cannot hold the tables";
                return ESP_E_UNSUPPORTED;
            }
        } else {
            hipError_t e = hipMalloc(&q, std::max<size_t>(b.size(), 16));
            if (e != hipSuccess) {
                msg = std::string("hipMalloc: ") + hipGetErrorString(e);
                return ESP_E_NOMEM;
            }
            allocs_.push_back(q);
        }
        hipError_t e = hipMemcpy(q, b.data(), b.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            msg = std::string("hipMemcpy: ") + hipGetErrorString(e);
            return ESP_E_DEVICE;
        }
        *dst[i] = q;
    }
    keep_.push_back(t);
    auto res = dev_.emplace(key, d);
    *out = &res.first->second;
    return ESP_OK;
}

int choose_tile(int n, int requested, long long target) {
    if (requested > 0) {
        // T >= 8 keeps every grid index inside at most 3 tiles per axis
        for (int d = std::min(requested, n); d >= 8; --d)
            if (n % d == 0) return d;
        for (int d = 8; d <= n; ++d)
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

std::vector<int> tile_candidates(int n, int P) {
    std::vector<int> out;
    for (int d = 8; d <= 16; ++d) {
        if (n % d) continue;
        const int E = d + P - 1 + (P & 1);
        const long long nb = (long long)(n / d) * (n / d) * (n / d);
        if ((long long)E * E * E * 8 + 2 * 12 * 17 * 8 <= kMaxLds && nb * 4 <= kMaxLds) out.push_back(d);
    }
    return out;
}

// The tile buffer also stages the scatter's output (particles in bin order
// and their caller indices) before the dealing pass writes the final order;
// the tiles are written later, by the spread.
size_t tiles_region(size_t tile_bytes, int64_t N, size_t rb) {
    const size_t stage = align256(N * 4 * rb) + align256(N * 4);
    return align256(std::max(tile_bytes, stage));
}

static_assert(kLocalCoefStride == kLocalMaxDegree + 1, "device table stride of the local polynomials");

void local_cells(const esp_params& p, int& lcs, int& R) {
    // the largest reach of rc in grid units along any index axis: rc n / d_d
    // for plane spacing d_d (rc/h_d along the finest axis of a box)
    const double rho = grid_rho(p) * p.L / cell_of(p).dmin;
    lcs = std::max(1, std::min(8, (int)std::floor(2.0 * p.tile / rho)));
    R = std::max(1, (int)std::ceil(rho * (1.0 + 1e-4) * lcs / p.tile));
}

static double halo_particles(int a, int R, int lcs, int T, int n, long long N) {
    const double edge = (double)(a + 2 * R) * T / lcs;  // grid units
    return (double)N / ((double)n * n * n) * edge * edge * edge;
}

int local_block(int lcs, int R, int T, int n, long long N, double limit) {
    for (int a = lcs; a > 1; --a)
        if (lcs % a == 0 && halo_particles(a, R, lcs, T, n, N) <= limit) return a;
    return 1;
}

size_t scratch_bytes(const esp_params& p, int64_t N) {
    const size_t rb = p.precision == 64 ? 8 : 4;
    const size_t nb = nbins(p), E = tile_edge(p), n = p.nf;
    size_t s = 0;
    s += align256(N * 4 * rb);                   // sorted
    s += align256(N * 4);                        // perm
    s += align256(N * 4);                        // rank
    s += align256(nb * npitems(N) * 4);          // hist
    s += align256((nb + 1) * 4);                 // bin_start
    s += align256(n * n * (n + 2) * rb);         // grid
    if (p.force_method == 1) s += align256(3 * n * n * (n + 2) * rb);  // gradient grids
    s += tiles_region(nb * E * E * E * rb, N, rb);  // tiles / staging of the scatter
    if (non_cubic(p)) s += align256((size_t)n * n * (n / 2 + 1) * rb);  // influence table
    if (p.local) {
        int lcs, R;
        local_cells(p, lcs, R);
        s += align256(N * 4 * rb);               // cpos
        s += align256(N * 4);                    // cidx
        s += align256((nb * lcs * lcs * lcs + 1) * 4);  // cstart
        s += align256(N * 4 * rb);               // loc
    }
    s += align256(kOutDoubles * 8);              // out
    return s;
}

SysScratch carve_scratch(unsigned char* base, const esp_params& p, int64_t N) {
    const size_t rb = p.precision == 64 ? 8 : 4;
    const size_t nb = nbins(p), E = tile_edge(p), n = p.nf;
    SysScratch s;
    size_t o = 0;
    s.sorted = base + o;
    o += align256(N * 4 * rb);
    s.perm = reinterpret_cast<int*>(base + o);
    o += align256(N * 4);
    s.rank = reinterpret_cast<int*>(base + o);
    o += align256(N * 4);
    s.hist = reinterpret_cast<int*>(base + o);
    o += align256(nb * npitems(N) * 4);
    s.bin_start = reinterpret_cast<int*>(base + o);
    o += align256((nb + 1) * 4);
    s.grid = base + o;
    o += align256(n * n * (n + 2) * rb);
    s.grad = nullptr;
    if (p.force_method == 1) {
        s.grad = base + o;
        o += align256(3 * n * n * (n + 2) * rb);
    }
    s.tiles = base + o;
    o += tiles_region(nb * E * E * E * rb, N, rb);
    s.p3 = nullptr;
    if (non_cubic(p)) {
        s.p3 = base + o;
        o += align256((size_t)n * n * (n / 2 + 1) * rb);
    }
    s.cpos = s.loc = nullptr;
    s.cidx = s.cstart = nullptr;
    if (p.local) {
        int lcs, R;
        local_cells(p, lcs, R);
        s.cpos = base + o;
        o += align256(N * 4 * rb);
        s.cidx = reinterpret_cast<int*>(base + o);
        o += align256(N * 4);
        s.cstart = reinterpret_cast<int*>(base + o);
        o += align256((nb * lcs * lcs * lcs + 1) * 4);
        s.loc = base + o;
        o += align256(N * 4 * rb);
    }
    s.out = reinterpret_cast<double*>(base + o);
    return s;
}

LaunchSet::~LaunchSet() {
    if (arena_) return;  // the arena's owner keeps its memory
    void* ps[] = {d_sys_,  d_pitems_, d_titems_, d_xitems_, d_planes_, d_fsys_, d_bsys_,
                  d_cols_, d_bpart_,  d_epart_,  d_lpart_,  d_litems_};
    for (void* p : ps)
        if (p) (void)hipFree(p);
}

esp_status LaunchSet::obtain(void** dev, size_t bytes, std::string& msg) {
    if (arena_) {
        *dev = arena_->take(bytes);
        if (!*dev) {
            msg = "the fixed scratch block cannot hold the launch lists";
            return ESP_E_UNSUPPORTED;
        }
        return ESP_OK;
    }
    if (*dev) (void)hipFree(*dev);
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, bytes);
    if (e != hipSuccess) {
        msg = std::string("hipMalloc: ") + hipGetErrorString(e);
        return ESP_E_NOMEM;
    }
    return ESP_OK;
}

template <class T>
esp_status LaunchSet::put(T** dev, size_t* cap, const std::vector<T>& v, std::string& msg) {
    if (v.size() > *cap || !*dev) {
        const size_t c = std::max<size_t>(v.size() + v.size() / 2, 16);
        esp_status st = obtain(reinterpret_cast<void**>(dev), c * sizeof(T), msg);
        if (st != ESP_OK) return st;
        *cap = c;
    }
    if (!v.empty()) {
        hipError_t e = hipMemcpyAsync(*dev, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, L_.stream);
        if (e != hipSuccess) {
            msg = std::string("hipMemcpyAsync: ") + hipGetErrorString(e);
            return ESP_E_DEVICE;
        }
    }
    return ESP_OK;
}

esp_status LaunchSet::build(const std::vector<SystemSlot>& systems, int prec, hipStream_t stream,
                            std::string& msg, int max_lanes) {
    const int rb = prec == 64 ? 8 : 4;
    const int nsys = (int)systems.size();
    hsys_.assign(nsys, SysDesc{});
    pitems_.clear();
    titems_.clear();
    xitems_.clear();
    planes_.clear();
    cols_.clear();
    groups_.clear();
    fgroups_.clear();
    fsys_.clear();
    bsys_.clear();
    litems_.clear();
    // bin work items by window width: one spread / gather launch per P (a
    // launch per further key, say tile edge, would serialise launches whose
    // tails leave the chip idle)
    std::vector<std::vector<int2>> titems_by_P(13);
    int nb_max = 1, nb_small_max = 1, n_eligible = 0;
    bool any_ik = false, any_local = false;
    for (int s = 0; s < nsys; ++s) {
        const SystemSlot& sl = systems[s];
        const esp_params& r = sl.prm;
        const ClassTables& ct = *sl.cls->host;
        SysDesc& d = hsys_[s];
        d.n = r.nf;
        d.P = r.P;
        d.N = (int)sl.N;
        d.T = r.tile;
        d.tiles1 = r.nf / r.tile;
        d.mT = (int)(((1 << 20) + d.T - 1) / d.T);
        d.mt1 = (int)(((1 << 20) + d.tiles1 - 1) / d.tiles1);
        d.E = tile_edge(r);
        d.degree = r.degree;
        d.inv_L = 1.0 / r.L;
        d.inv_Ly = 1.0 / r.Ly;
        d.inv_Lz = 1.0 / r.Lz;
        d.side[0] = r.L;
        d.side[1] = r.Ly;
        d.side[2] = r.Lz;
        d.nside[0] = (double)r.nf / r.L;
        d.nside[1] = (double)r.nf / r.Ly;
        d.nside[2] = (double)r.nf / r.Lz;
        d.tilt = tilted(r) ? 1 : 0;
        d.lay = r.Ly / r.L;  // h_y / h_x
        d.laz = r.Lz / r.L;
        {
            const Cell c = cell_of(r);
            d.ixy = c.ixy;
            d.ixz = c.ixz;
            d.iyz = c.iyz;
            d.mxy = r.xy / r.L;
            d.mxz = r.xz / r.L;
            d.myz = r.yz / r.L;
            const bool tilt = tilted(r);
            d.ikx = tilt ? 1.0 : d.inv_L;
            d.iky = tilt ? 1.0 : d.inv_Ly;
            d.ikz = tilt ? 1.0 : d.inv_Lz;
        }
        d.p3 = sl.scr.p3;
        d.pscale = r.nf / r.L;
        d.s0 = non_cubic(r) ? r.s0 : ct.s0_ref * r.nf / r.L;
        d.wmax3 = ct.wmax3;
        d.TS = sl.cls->TS;
        d.Tphi = sl.cls->Tphi;
        d.poly = sl.cls->poly;
        d.tw = sl.cls->tw;
        d.pos = sl.pos;
        d.q = sl.q;
        d.phi = sl.phi;
        d.F = sl.F;
        d.sorted = sl.scr.sorted;
        d.perm = sl.scr.perm;
        d.rank = sl.scr.rank;
        d.hist = sl.scr.hist;
        d.bin_start = sl.scr.bin_start;
        d.grid = sl.scr.grid;
        d.grad = sl.scr.grad;
        d.ik = r.force_method == 1;
        any_ik = any_ik || d.ik;
        d.local = r.local == 1;
        any_local = any_local || d.local;
        if (d.local) {
            local_cells(r, d.lcs, d.lR);
            d.lsa = local_block(d.lcs, d.lR, d.T, d.n, d.N, kLocalHaloTarget);
            const int nsb = d.lcs / d.lsa, nb = d.tiles1 * d.tiles1 * d.tiles1;
            d.litem_off = (int)litems_.size();
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < nsb * nsb * nsb; ++k) litems_.push_back(make_int2(s, b * nsb * nsb * nsb + k));
            d.nlitem = (int)litems_.size() - d.litem_off;
            const double rho = grid_rho(r);
            d.ldeg = ct.ldeg;
            d.lsT = (double)d.lcs / d.T;
            d.lrho2 = rho * rho;
            d.lcoef = sl.cls->lcoef;
            d.cpos = sl.scr.cpos;
            d.cidx = sl.scr.cidx;
            d.cstart = sl.scr.cstart;
            d.loc = sl.scr.loc;
            if (d.lR > d.tiles1 * d.lcs) {  // one periodic wrap per axis reaches every image
                msg = "local-part stencil wider than the box";
                return ESP_E_UNSUPPORTED;
            }

        }
        d.tiles = sl.scr.tiles;
        d.out = sl.scr.out;
        d.seed = sl.seed;
        d.drift = sl.drift;
        d.step = 0;
        d.pitem_off = (int)pitems_.size();
        for (int c = 0; c < d.N; c += kParticleChunk) pitems_.push_back(make_int2(s, c));
        d.npitem = (int)pitems_.size() - d.pitem_off;
        const int nb = d.tiles1 * d.tiles1 * d.tiles1;
        d.small = d.N <= kSmallMaxN && nb <= kSmallMaxBins;
        if (d.small) ++n_eligible;
        for (int t = 0; t < nb; ++t) titems_by_P[r.P].push_back(make_int2(s, t));
        if (!fft_size_supported(r.nf)) {
            msg = "no FFT kernels for this grid size";
            return ESP_E_UNSUPPORTED;
        }
        if (fft_plane_lds(r.nf, prec) > kMaxLds) {
            msg = "grid too large for the LDS-resident plane FFT at this precision";
            return ESP_E_UNSUPPORTED;
        }
    }
    // one block per system bins a system faster than the chunked kernels when
    // enough systems share the launch to fill the GPU, or when the system is
    // small enough that one launch beats the chunked path's five (the
    // particle order within a bin, which is all the path changes, affects no
    // result)
    // A block's binning time grows with its system's size, so with many
    // systems a system above three times the median size of the candidates (and
    // above kSmallAlwaysN) takes the chunked path, which runs beside the
    // one-block launch, instead of finishing long after the other blocks; in
    // FP32 so does a system too large to keep its particles in registers
    // (kSmallKeep), when the chunked path runs anyway.
    int n_split = kSmallMaxN;
    if (n_eligible >= kSmallMinSystems) {
        std::vector<int> ns;
        for (const SysDesc& d : hsys_)
            if (d.small) ns.push_back(d.N);
        std::nth_element(ns.begin(), ns.begin() + ns.size() / 2, ns.end());
        n_split = std::max(kSmallAlwaysN, 3 * ns[ns.size() / 2]);
        const bool chunked = std::any_of(ns.begin(), ns.end(), [&](int N) { return N > n_split; });
        if (prec == 32 && chunked) n_split = std::min(n_split, std::max(kSmallAlwaysN, kSmallKeep * 1024));
    }
    int scan_rows_fused = 1;
    for (int s = 0; s < nsys; ++s) {
        SysDesc& d = hsys_[s];
        const int nb = d.tiles1 * d.tiles1 * d.tiles1;
        if (n_eligible < kSmallMinSystems && d.N > kSmallAlwaysN) d.small = 0;
        if (d.N > n_split) d.small = 0;
        if (d.small) {
            bsys_.push_back(make_int2(s, 0));
            nb_small_max = std::max(nb_small_max, nb);
        } else {
            nb_max = std::max(nb_max, nb);
            if (nb > kScanRowsMax || d.npitem > kScanRowsMax) scan_rows_fused = 0;
        }
    }
    // FFT work items grouped by (grid size, path): one launch per group and
    // pass, largest grids first (dealt to the pipeline lanes in that order).
    // Systems that ask for the one-block transform
    // and whose half spectrum fits in LDS take it; their energy partial goes
    // to one slot after the x-column items.
    // (ik systems apart: the x pass of AD systems up to n = 64 (FP32) keeps
    // each column in registers, k_fft_x_reg, 64 columns per block)
    std::map<std::array<int, 3>, std::vector<int>> by_n;
    for (int s = 0; s < nsys; ++s) {
        const int n = hsys_[s].n;
        const int fused = systems[s].prm.fft_passes == 1 && !hsys_[s].ik && !hsys_[s].p3 &&
                          fft_fused_lds(n, prec) <= kMaxLds;
        by_n[{n, fused, hsys_[s].ik ? 1 : 0}].push_back(s);
        hsys_[s].fin_fft = !fused;  // the plane-pass FFT's last kernel finalizes the energy
    }
    std::vector<int> fused_sys;
    for (auto git = by_n.rbegin(); git != by_n.rend(); ++git) {
        const auto& kv = *git;
        const int n = kv.first[0], hs = n / 2 + 1;
        FftGroup fg{};
        fg.n = n;
        fg.fused = kv.first[1];
        fg.xreg = !fg.fused && !kv.first[2] && fft_x_in_registers(n, prec);
        const int C = fg.xreg ? kXRegColumns : fft_x_columns(prec);
        fg.plane_off = (int)planes_.size();
        fg.col_off = (int)cols_.size();
        fg.sys_off = (int)fsys_.size();
        for (int s : kv.second) {
            // x-planes of every system (the diagnostic fold walks them all)
            for (int x = 0; x < n; ++x) planes_.push_back(make_int2(s, x));
            if (fg.fused) {
                fsys_.push_back(make_int2(s, 0));
                fused_sys.push_back(s);
                continue;
            }
            SysDesc& d = hsys_[s];
            d.col_off = (int)cols_.size();
            for (int c0 = 0; c0 < n * hs; c0 += C) cols_.push_back(make_int4(s, c0, std::min(C, n * hs - c0), 0));
            d.ncol = (int)cols_.size() - d.col_off;
        }
        fg.plane_count = (int)planes_.size() - fg.plane_off;
        fg.col_count = (int)cols_.size() - fg.col_off;
        fg.sys_count = (int)fsys_.size() - fg.sys_off;
        fgroups_.push_back(fg);
    }
    // lanes: FFT groups, largest grid first, each to the lane with the least
    // work so far; work = FFT (systems x n^3 log2 n) plus spread and gather
    // (particles), weighted as measured on MI355X (about 3.1e-6 and 1.0e-4
    // microseconds per unit)
    lanes_ = std::max(1, std::min<int>(max_lanes, (int)fgroups_.size()));
    std::vector<int> sys_lane(nsys, 0);
    {
        std::vector<double> load(lanes_, 0.0);
        for (FftGroup& fg : fgroups_) {
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            fg.lane = l;
            double w = 0.0;
            const int2* it = fg.fused ? &fsys_[fg.sys_off] : &planes_[fg.plane_off];
            const int step = fg.fused ? 1 : fg.n;  // a system's planes are consecutive
            const int cnt = fg.fused ? fg.sys_count : fg.plane_count;
            for (int k = 0; k < cnt; k += step) {
                const int s = it[k].x;
                sys_lane[s] = l;
                w += 3.1e-6 * std::pow((double)fg.n, 3) * std::log2((double)fg.n) + 1.0e-4 * hsys_[s].N;
            }
            load[l] += w;
        }
    }
    sys_lane_ = sys_lane;
    const int n_eslots = (int)cols_.size() + (int)fused_sys.size();
    for (size_t k = 0; k < fused_sys.size(); ++k) {
        SysDesc& d = hsys_[fused_sys[k]];
        d.col_off = (int)cols_.size() + (int)k;
        d.ncol = 1;
    }
    for (int lane = 0; lane < lanes_; ++lane) {
        for (int P = 4; P <= 12; ++P) {
            std::vector<int2> items;  // the lane's bins of window width P
            for (const int2& it : titems_by_P[P])
                if (sys_lane[it.x] == lane) items.push_back(it);
            if (items.empty()) continue;
            Group g;
            g.P = P;
            g.lane = lane;
            int E = 0;
            for (const int2& it : items) E = std::max(E, hsys_[it.x].E);
            // XCD order: runs of consecutive bins of one system (neighbours,
            // which share halo rows), at most ceil(bins / (4 kXcds)) long so
            // that a large system spreads over every XCD, largest first to
            // the XCD with the least work so far (work ~ particles plus 40
            // per bin for its tile), so that the XCDs finish together and a
            // run's halos are fetched once into one L2
            const int cap = std::max<int>(1, (int)((items.size() + 4 * kXcds - 1) / (4 * kXcds)));
            struct Piece {
                int s, t0, nb;
                double w;
            };
            std::vector<Piece> pieces;
            for (size_t k = 0; k < items.size();) {
                const int s = items[k].x;
                size_t e = k;
                while (e < items.size() && items[e].x == s) ++e;  // the system's bins
                const SysDesc& d = hsys_[s];
                const int nb = (int)(e - k);
                const double per_bin = (double)d.N / nb + 40.0;
                for (int t0 = 0; t0 < nb; t0 += cap) {
                    const int m = std::min(cap, nb - t0);
                    pieces.push_back({s, items[k].y + t0, m, per_bin * m});
                }
                k = e;
            }
            std::stable_sort(pieces.begin(), pieces.end(), [](const Piece& a, const Piece& b) { return a.w > b.w; });
            std::vector<std::vector<int2>> runs(kXcds);
            std::vector<double> load(kXcds, 0.0);
            for (const Piece& pc : pieces) {
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[x] += pc.w;
                for (int t = 0; t < pc.nb; ++t) runs[x].push_back(make_int2(pc.s, pc.t0 + t));
            }
            size_t per = 0;
            for (const auto& r : runs) per = std::max(per, r.size());
            g.off = (int)xitems_.size();
            g.count = (int)(per * kXcds);
            for (auto& r : runs) {
                r.resize(per, make_int2(-1, -1));
                xitems_.insert(xitems_.end(), r.begin(), r.end());
            }
            // spread: the accumulators (32-bit fixed point for FP32 windows up
            // to P = 6, else 64-bit fixed point or double), then the window
            // coefficients; gather: the potential tile, the coefficients and
            // their derivatives, the tile's E^2 row offsets
            g.lds_spread = E * E * E * (prec == 32 && P <= 6 ? 4 : 8) + kCoefBytes;
            g.lds_gather = ((E * E * E * rb + 15) & ~15) + gather_coef_bytes(P, (int)rb) + E * E * 4;
            if (g.lds_spread > kMaxLds || g.lds_gather > kMaxLds) {
                msg = "bin tile (T+P)^3 exceeds LDS; reduce tile";
                return ESP_E_UNSUPPORTED;
            }
            groups_.push_back(g);
        }
    }
    for (int P = 4; P <= 12; ++P) titems_.insert(titems_.end(), titems_by_P[P].begin(), titems_by_P[P].end());
    L_.prec = prec;
    L_.nsys = nsys;
    L_.any_local = any_local;
    L_.any_fin_kernel = 0;
    for (const SysDesc& d : hsys_) L_.any_fin_kernel = L_.any_fin_kernel || !d.fin_fft;
    // LDS staging of a bin's halo for the local pass: the expected particle
    // count of the largest halo with 30% headroom (a bin whose halo holds more
    // takes the global-memory path), within 64 KB
    L_.local_cap = 0;
    L_.local_cells = 0;
    L_.local_deg = 0;
    if (any_local) {
        double want = 0.0;
        for (const SysDesc& d : hsys_) {
            if (!d.local) continue;
            const int W = d.lsa + 2 * d.lR;
            L_.local_cells = std::max(L_.local_cells, W * W * W);
            want = std::max(want, halo_particles(d.lsa, d.lR, d.lcs, d.T, d.n, d.N));
        }
        const int vb = 4 * rb;
        const int capmax = (65536 - (L_.local_cells + 1) * 4) / vb;
        const int cap = ((int)(1.3 * want) + 64 + 63) / 64 * 64;
        L_.local_cap = std::max(64, std::min(cap, capmax));
        for (const SysDesc& d : hsys_)
            if (d.local) L_.local_deg = std::max(L_.local_deg, d.ldeg);
    }
    L_.stream = stream;
    L_.n_pitems = (int)pitems_.size();
    L_.n_titems = (int)titems_.size();
    L_.n_planes = (int)planes_.size();
    L_.n_cols = (int)cols_.size();
    L_.hist_lds = nb_max * 4;
    L_.any_ik = any_ik;
    L_.scan_rows_fused = scan_rows_fused;
    L_.n_small = (int)bsys_.size();
    L_.n_large = nsys - L_.n_small;
    L_.small_lds = (nb_small_max * 32 + 2 * (nb_small_max + 1) + 2 * kSmallRounds) * 4;
    if (L_.hist_lds > kMaxLds) {
        msg = "too many bins per system; raise tile";
        return ESP_E_UNSUPPORTED;
    }
    esp_status st;
    if ((st = put(&d_sys_, &cap_sys_, hsys_, msg)) != ESP_OK) return st;
    if ((st = put(&d_pitems_, &cap_pitems_, pitems_, msg)) != ESP_OK) return st;
    if ((st = put(&d_titems_, &cap_titems_, titems_, msg)) != ESP_OK) return st;
    if ((st = put(&d_xitems_, &cap_xitems_, xitems_, msg)) != ESP_OK) return st;
    if ((st = put(&d_planes_, &cap_planes_, planes_, msg)) != ESP_OK) return st;
    if ((st = put(&d_cols_, &cap_cols_, cols_, msg)) != ESP_OK) return st;
    if ((st = put(&d_fsys_, &cap_fsys_, fsys_, msg)) != ESP_OK) return st;
    if ((st = put(&d_bsys_, &cap_bsys_, bsys_, msg)) != ESP_OK) return st;
    if ((st = put(&d_litems_, &cap_litems_, litems_, msg)) != ESP_OK) return st;
    // partial sums are written before they are read: capacity only
    auto reserve = [&](double** dev, size_t* cap, size_t need) {
        if (need <= *cap && *dev) return ESP_OK;
        const size_t c = std::max<size_t>(need + need / 2, 16);
        esp_status st = obtain(reinterpret_cast<void**>(dev), c * sizeof(double), msg);
        if (st != ESP_OK) return st;
        *cap = c;
        return ESP_OK;
    };
    if ((st = reserve(&d_bpart_, &cap_bpart_, 4 * pitems_.size())) != ESP_OK) return st;
    if ((st = reserve(&d_epart_, &cap_epart_, (size_t)n_eslots)) != ESP_OK) return st;
    if ((st = reserve(&d_lpart_, &cap_lpart_, litems_.size())) != ESP_OK) return st;
    L_.sys = d_sys_;
    L_.pitems = d_pitems_;
    L_.titems = d_titems_;
    L_.xitems = d_xitems_;
    L_.planes = d_planes_;
    L_.cols = d_cols_;
    L_.fsys = d_fsys_;
    L_.bsys = d_bsys_;
    L_.bpart = d_bpart_;
    L_.epart = d_epart_;
    L_.lpart = d_lpart_;
    L_.litems = d_litems_;
    L_.n_litems = (int)litems_.size();
    return ESP_OK;
}

void LaunchSet::set_io(int s, const void* pos, const void* q, void* phi, void* F) {
    SysDesc& d = hsys_[s];
    d.pos = pos;
    d.q = q;
    d.phi = phi;
    d.F = F;
}

esp_status LaunchSet::upload_descriptors(std::string& msg) { return put(&d_sys_, &cap_sys_, hsys_, msg); }

}  // namespace esp
