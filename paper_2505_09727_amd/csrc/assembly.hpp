// Assembly of launch sets: per-system scratch layout, device copies of the
// table classes, and the descriptor / work-item lists of a set of systems.
// Shared by static plans (one set built once) and the server (rebuilt when
// the active set changes).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "esp.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace esp {

// Device memory handed out from one block the caller owns (no allocation):
// 256-byte aligned pieces, in order, until the block is used up.
struct FixedBlock {
    unsigned char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    void* take(size_t bytes) {
        const size_t o = (used + 255) & ~size_t(255);
        if (o > cap || bytes > cap - o) return nullptr;
        used = o + bytes;
        return base + o;
    }
};

// Device copy of one table class (owned by a TableStore).
struct DeviceClass {
    const ClassTables* host = nullptr;
    void* TS = nullptr;
    void* Tphi = nullptr;
    void* poly = nullptr;
    void* tw = nullptr;
    void* lcoef = nullptr;  // local-part polynomials A then B
};

// Uploads each table class once per precision and keeps it until destroyed.
class TableStore {
  public:
    ~TableStore();
    // Device tables for resolved params (uploads on first use).
    esp_status get(const esp_params& p, const DeviceClass** out, std::string& msg);
    // Take device memory from `a` instead of allocating it (before any get).
    void set_arena(FixedBlock* a) { arena_ = a; }

  private:
    FixedBlock* arena_ = nullptr;
    std::map<std::pair<const ClassTables*, int>, DeviceClass> dev_;
    std::vector<std::shared_ptr<const ClassTables>> keep_;
    std::vector<void*> allocs_;
};

// Bin edge: a divisor of n in [8, 16] giving at least `target` bins when
// possible (requested > 0 rounds a caller's choice down to a divisor >= 8).
int choose_tile(int n, int requested, long long target);
// Bin edges an autotuner may try for grid n and window P: divisors of n in
// [8, 16] whose spread tile and bin histogram fit in LDS.
std::vector<int> tile_candidates(int n, int P);

// Scratch of one system, carved from one block of device memory.
struct SysScratch {
    void* sorted;
    int* perm;
    int* rank;
    int* hist;
    int* bin_start;
    void* grid;
    void* grad;   // ik: three more grids (null otherwise)
    void* tiles;
    void* cpos;   // local part only (null otherwise): sub-cell ordered copy,
    int* cidx;    // its sorted indices,
    int* cstart;  // sub-cell starts,
    void* loc;    // and the per-particle local results
    void* p3;     // orthorhombic box only: the influence table, n x n x (n/2 + 1)
    double* out;
};
// Host FP64 values converted to the plan precision (bytes).
std::vector<unsigned char> to_prec(const std::vector<double>& v, int prec);
// Whether resolved params describe a non-cubic box.
inline bool non_cubic(const esp_params& p) { return p.Ly != p.L || p.Lz != p.L || tilted(p); }
// Local part: sub-cells per bin side and stencil radius for resolved params.
void local_cells(const esp_params& p, int& lcs, int& R);
// Local part: sub-cells per side of one work item's block (a divisor of lcs
// whose halo, (a + 2R)^3 sub-cells, is expected to hold at most `limit`
// particles; 1 if none does) for N particles on grid n.
int local_block(int lcs, int R, int T, int n, long long N, double limit);
size_t scratch_bytes(const esp_params& p, int64_t N);
SysScratch carve_scratch(unsigned char* base, const esp_params& p, int64_t N);

// One system placed in a launch set.
struct SystemSlot {
    esp_params prm;
    int64_t N = 0;
    const DeviceClass* cls = nullptr;
    SysScratch scr{};
    const void* pos = nullptr;
    const void* q = nullptr;
    void* phi = nullptr;
    void* F = nullptr;
    unsigned long long seed = 0;  // serving drift stream
    float drift = 0.0f;
};

// Pipeline lanes of a launch set with several FFT grid-size groups: the
// plan's stream and two side streams, which (with the binning's side stream
// reused) fit the 4 hardware queues a process gets by default.
constexpr int kLanes = 3;

// Host and device copies of a launch set.
class LaunchSet {
  public:
    ~LaunchSet();
    // Build descriptors and work lists for `systems` (same precision) and
    // upload them on `stream`. Device arrays grow as needed.
    // max_lanes caps the pipeline lanes (1 for a caller that launches every
    // group on one stream, as the server does).
    esp_status build(const std::vector<SystemSlot>& systems, int prec, hipStream_t stream, std::string& msg,
                     int max_lanes = kLanes);
    // Re-point the particle arrays of system s (no upload).
    void set_io(int s, const void* pos, const void* q, void* phi, void* F);
    // Serving: drift step of system s for the next drift launch (0: none).
    void set_step(int s, int step) { hsys_[s].step = step; }
    // Upload the descriptors after set_io / set_step.
    esp_status upload_descriptors(std::string& msg);
    const Launch& launch() const { return L_; }
    // Stream of later launches and uploads.
    void set_stream(hipStream_t stream) { L_.stream = stream; }
    // Take device memory from `a` instead of allocating it (before build).
    void set_arena(FixedBlock* a) { arena_ = a; }
    const std::vector<Group>& groups() const { return groups_; }
    // Pipeline lanes: the FFT grid-size groups, and with them their systems,
    // are dealt to `lanes()` lanes (largest first, each to the lane with the
    // least work so far), and a step may run each lane's spread, FFT passes
    // and gather on a stream of its own. 1 when there is one FFT group.
    int lanes() const { return lanes_; }
    int lane_of(int s) const { return sys_lane_[s]; }
    const std::vector<FftGroup>& fft_groups() const { return fgroups_; }
    int nsys() const { return (int)hsys_.size(); }
    const SysDesc& desc(int s) const { return hsys_[s]; }

  private:
    template <class T>
    esp_status put(T** dev, size_t* cap, const std::vector<T>& v, std::string& msg);
    // Device memory of `bytes` for a launch-set array (allocated, or from the arena).
    esp_status obtain(void** dev, size_t bytes, std::string& msg);
    FixedBlock* arena_ = nullptr;
    Launch L_{};
    std::vector<Group> groups_;
    std::vector<FftGroup> fgroups_;
    int lanes_ = 1;
    std::vector<int> sys_lane_;
    std::vector<SysDesc> hsys_;
    std::vector<int2> pitems_, titems_, xitems_, planes_, fsys_, bsys_, litems_;
    std::vector<int4> cols_;
    SysDesc* d_sys_ = nullptr;
    int2 *d_pitems_ = nullptr, *d_titems_ = nullptr, *d_xitems_ = nullptr, *d_planes_ = nullptr, *d_fsys_ = nullptr, *d_bsys_ = nullptr,
         *d_litems_ = nullptr;
    int4* d_cols_ = nullptr;
    double *d_bpart_ = nullptr, *d_epart_ = nullptr, *d_lpart_ = nullptr;
    size_t cap_sys_ = 0, cap_pitems_ = 0, cap_titems_ = 0, cap_xitems_ = 0, cap_planes_ = 0, cap_fsys_ = 0, cap_bsys_ = 0, cap_cols_ = 0,
           cap_bpart_ = 0, cap_epart_ = 0, cap_lpart_ = 0, cap_litems_ = 0;
};

constexpr int kMaxLds = 160 * 1024;

}  // namespace esp
