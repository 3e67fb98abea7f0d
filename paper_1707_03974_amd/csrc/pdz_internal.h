// Internal declarations shared by the pdz host runtime and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pdz.h"

namespace pdz {

constexpr int kMaxSites = 32;
constexpr int kBinomStride = kMaxSites + 1;          // C[i * 33 + m], i, m in [0, 32]
constexpr uint32_t kTargetBits = 24;                   // hop-table entry: target | coef << 24
constexpr uint32_t kTargetMask = (1u << kTargetBits) - 1u;
constexpr int kMaxCoef = 256;                          // distinct signed hop amplitudes
constexpr uint32_t kBadRank = 0xFFFFFFFFu;

// Device error word bits.
constexpr uint32_t kErrRankInput = 1u;     // pdz_rank: popcount or width mismatch
constexpr uint32_t kErrUnrankInput = 2u;   // pdz_unrank: rank out of range
constexpr uint32_t kErrTable = 4u;         // hop-table build: a target failed to rank
constexpr uint32_t kErrNonFinite = 8u;     // Lanczos: non-finite scalar

// One bond as the kernels see it.
struct BondDev {
    uint32_t mask;      // (1<<i) | (1<<j)
    uint32_t between;   // bits strictly between min(i,j) and max(i,j)
    int32_t coef_pos;   // index of -t in the coefficient table (even number of passed operators)
    int32_t coef_neg;   // index of +t (odd number)
};

// Bank-conflict-free gather schedule of the down pass over one sector
// (pdz_sched.cpp): per wave of 64 columns S steps (a multiple of 4), the
// first B of them (a multiple of 4) with the smaller hop magnitude mag0, the
// rest with mag1.  A step is a 16-bit entry per lane: the byte address of its
// target in a row plane of kSchedPlane words (the last 32 are zeros), bit 0
// set when the lane adds -mag.  Word i of a lane holds steps 2i (low half)
// and 2i + 1; a lane's words lie four at a time, words[off[w] + q * 256 +
// lane * 4 + j] = word 4q + j of wave w (a last pair: lane * 2 + j);
// meta[2 w] = off[w], meta[2 w + 1] = S | B << 16.  words == NULL: no
// schedule.
constexpr uint32_t kSchedPlane = 13312;   // words per plane: sectors of at most 13280 states
constexpr int kSchedMaxSteps = 64;        // a longer schedule is not built
struct DownSchedule {
    uint32_t* words = nullptr;
    uint32_t* meta = nullptr;    // per wave: word offset, S | B << 16
    uint32_t plane = 0;
    double mag0 = 0.0, mag1 = 0.0;
    size_t nwords = 0;
};

// Per-spin sector tables on the device (ELL layout, hop slot major).
struct SectorTables {
    uint64_t D = 0;             // sector size C(N, n)
    int n = 0;                  // electrons of this spin
    int max_hops = 0;           // most hops out of one state
    uint64_t total_hops = 0;    // hops summed over the sector
    uint32_t* states = nullptr; // D occupation strings (backward map of each rank)
    uint8_t* count = nullptr;   // D hop counts
    uint32_t* ell = nullptr;    // max_hops * D entries: ell[h * D + s] = target | coef << 24
    uint16_t* ell16 = nullptr;  // target | coef << tbits16 when that fits 16 bits, slot-pair layout:
                                // slot h of state s at ((h / 2) * D + s) * 2 + h % 2
    int tbits16 = 0;            // target bits of a 16-bit entry (0: no 16-bit table)
    DownSchedule sched;         // gather schedule for a down pass over this sector
};

}  // namespace pdz

namespace pdz {
struct KSpace;   // momentum-space sector tables (k_kspace.hip)
struct ParSpace; // inversion-parity tables (k_parity.hip)
// H.v launch plan for one precision (0 = automatic choice).
struct HvPlan {
    int down = 0;    // 1: one row per group, hop table loaded up front; 2: one row, table in a loop;
                     // 3: two rows per group, table in a loop
    int up_cw = 0;   // up-pass chunk width in columns
    int up = 0;      // 1: hops of a row loaded in batches of 8; 2: all hops of a row loaded up front
    int map = 0;     // up-pass tile order: 1 XCD-aware chunk pairs, 2 chunk-major, 3 XCD-aware single chunks
};
}  // namespace pdz

struct pdz_problem_s {
    int device = 0;
    int N = 0, n_up = 0, n_dn = 0, n_bonds = 0;
    double U = 0.0;
    std::vector<pdz_bond> bonds;
    uint64_t D = 0, nnz = 0;
    pdz::SectorTables up, dn;
    bool same_sector = false;            // dn tables alias the up tables
    uint32_t* d_binom = nullptr;         // 33 x 33 binomial table
    pdz::BondDev* d_bonds = nullptr;
    std::vector<double> coef_host;       // signed hop amplitudes
    double* d_coef64 = nullptr;
    float* d_coef32 = nullptr;
    int hv_path = 0;                     // 0 tables, 1 on the fly, 2 momentum space (ks), 3 parity (par)
    pdz::KSpace* ks = nullptr;           // momentum-space sector (Sec. IV.A), else NULL
    pdz::ParSpace* par = nullptr;        // inversion-parity subspace (Sec. IV.B; hv_path 3), else NULL
    pdz::HvPlan plan[2];                 // per pdz_dtype
};

namespace pdz {

// Error reporting (thread-local message).
pdz_status fail(pdz_status code, const std::string& msg);
pdz_status ok();
pdz_status hip_fail(hipError_t e, const char* what);
#define PDZ_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return pdz::hip_fail(e_, #call); \
    } while (0)

// Per-device context: error word and small scratch.
struct DeviceCtx {
    int device = -1;
    uint32_t* err = nullptr;       // device error word
    uint32_t* binom = nullptr;     // 33 x 33 binomial table
    int cu_count = 0;
    size_t lds_per_block = 0;
};
pdz_status device_ctx(DeviceCtx** out);

// SplitMix64, output r of the generator seeded with `seed`, as a double in [-1, 1).
__device__ inline double splitmix_uniform(uint64_t seed, uint64_t r) {
    uint64_t z = seed + (r + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

// One element of the Lanczos three-term recurrence on unnormalised vectors,
// q_{k+1} = a (hd + hu) - b q_k - c q_{k-1} (hd, hu: the two parts of H q_k),
// in FP64 with a fixed multiply-add order and one rounding to T.  Every kernel
// that forms a Lanczos vector uses it, so a vector formed by a fused pass and
// the same vector regenerated by the separate update are equal bit for bit.
template <typename T>
__device__ __forceinline__ T lanczos_recurrence(T hd, T hu, T qk, T qkm1, double a, double b, double c) {
    const double hq = (double)hd + (double)hu;
    const double t = fma(b, (double)qk, c * (double)qkm1);
    return (T)fma(a, hq, -t);
}

// Host helpers.
void binomial_table(std::vector<uint32_t>& C);   // Pascal's rule, 33 x 33
uint64_t binom(int n, int k);

// Kernel launchers (defined in the .hip files).
pdz_status launch_rank(const uint32_t* d_binom, int N, int n, const uint32_t* bits, uint64_t count,
                       uint32_t* ranks, uint32_t* err, hipStream_t s);
pdz_status launch_unrank(const uint32_t* d_binom, int N, int n, const uint32_t* ranks, uint64_t count,
                         uint32_t* bits, uint32_t* err, hipStream_t s);
pdz_status build_sector_tables(const uint32_t* d_binom, int N, int n, const BondDev* d_bonds, int nb,
                               SectorTables* st, uint32_t* err, hipStream_t s);
pdz_status build_compact_table(SectorTables* st, int ncoef, hipStream_t s);
// Down-pass gather schedule of a sector (host colouring; no schedule when the
// sector has more than kSchedPlane - 32 states or more than two hop magnitudes).
pdz_status build_down_schedule(const SectorTables& t, const std::vector<double>& coef, DownSchedule* out,
                               hipStream_t s);
void free_down_schedule(DownSchedule* sc);
pdz_status hv_prepare();   // per-device kernel attributes, called once outside any capture
pdz_status batch_prepare();   // the same for the batched H.v kernels
pdz_status kspace_prepare();  // the same for the momentum-space H.v kernels
pdz_status parity_prepare();  // the same for the parity H.v kernels
void kspace_free(KSpace* ks);
void parity_free(ParSpace* q);
// y = H x on an inversion-parity subspace; dotp (optional) receives
// parity_dot_count partial sums of x . y, whose total is x . y
pdz_status launch_hvp(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                      const int* skip, double* dotp = nullptr);
// partial sums launch_hvp writes to dotp; 0 when it cannot write them
int parity_dot_count(const pdz_problem_s* p, pdz_dtype dt);
// whether the parity down pass of the full rows runs gather-scheduled
bool parity_sched_down(const pdz_problem_s* p, pdz_dtype dt);
// y = H x on a momentum-space problem (every pass at once; no split form)
pdz_status launch_hvk(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                      const int* skip);
// Candidate plans for this problem and precision; the first is the default.
// Where the down sector has a gather schedule the tuner's set holds only the
// scheduled down family (one summation order); every = true adds the looped
// family, which a caller may still select.
std::vector<HvPlan> hv_candidates(const pdz_problem_s* p, pdz_dtype dt, bool every = false);
bool hv_plan_valid(const pdz_problem_s* p, pdz_dtype dt, const HvPlan& plan);
// passes: kPassDown | kPassUp for y = H x; one bit alone launches only that
// pass of the table path (the down pass writes y, the up pass adds onto it).
// split (table path only): the up term goes to split->z instead of being
// added to y, and each pass writes per-work-group partial sums of x . (its
// output) to dotp_dn / dotp_up (counts from hv_dot_counts); the sums in index
// order give x . (H x) = sum(dotp_dn) + sum(dotp_up).
constexpr unsigned kPassDown = 1u, kPassUp = 2u;
struct HvSplit {
    void* z = nullptr;          // D elements of the same precision as y
    double* dotp_dn = nullptr;
    double* dotp_up = nullptr;
    // Fused Lanczos recurrence in the down pass (fq2 != NULL; down pass only,
    // and hv_fused_available): the rows it stages are q_{k+1} formed from
    // y (down part of H q_k, overwritten with the down part of H q_{k+1}),
    // fz (up part of H q_k), fq1 = q_k and fq2 = q_{k-1} (overwritten with
    // q_{k+1}; copied to slot k + 1 of fkeep when set) with the scalars at
    // index *fkidx; fnorm receives one partial |q_{k+1}|^2 per work group.
    const void* fq1 = nullptr;
    void* fq2 = nullptr;
    const void* fz = nullptr;
    void* fkeep = nullptr;
    uint64_t fkeep_ld = 0;
    int fkeep_cap = 0;
    const double* falpha = nullptr;
    const double* fbeta = nullptr;
    const double* fsc = nullptr;
    const int* fkidx = nullptr;
    double* fnorm = nullptr;
};
bool hv_fused_available(const pdz_problem_s* p, pdz_dtype dt);
// Parity H.v by passes (kPassDown: the down pass, with the recurrence when
// sp->fq2 is set; kPassUp: the up pass and the palindromic rows, with x . y
// partials in sp->dotp_up).  Its parts stay in y: sp->z, dotp_dn and fz must
// be null.
pdz_status launch_hvp_split(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                            const int* skip, unsigned passes, const HvSplit* sp);
// |q_{k+1}|^2 partials the fused parity down pass writes to fnorm; 0 when
// the problem has no fused form
int parity_fused_norms(const pdz_problem_s* p, pdz_dtype dt);
// The scheduled down pass over explicit row groups (k_hv.hip): the full rows
// of a parity subspace (every down string, in the column order whose hops
// `sched` was built from).  Group g: gnr[g] (1..R) rows of D_dn elements,
// consecutive from element goff[g]; grp_up[g * R + r] the up string of its
// row r (0 past its rows); col_dn[c] the down string of column c.
struct SchedGroups {
    const DownSchedule* sched = nullptr;
    uint64_t D_dn = 0;
    double U = 0.0;
    const uint32_t* grp_up = nullptr;
    const uint32_t* col_dn = nullptr;
    const uint64_t* goff = nullptr;
    const uint8_t* gnr = nullptr;
    uint64_t ngroups = 0;
    int R = 1;   // 1 to 3 (FP64: 1); with R = 1 every group is one row and gnr is not read
};
// y = diagonal + down hops over the groups' rows (fuse == NULL), or, with
// fuse->fq2 set, q_{k+1} formed from y (the whole H q_k, fuse->fz NULL), q_k
// and q_{k-1} as in HvSplit, staged, and the down part of H q_{k+1} written
// to y; one |q_{k+1}|^2 partial per work group in fuse->fnorm.
pdz_status launch_sched_groups(const SchedGroups& g, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                               const int* skip, const HvSplit* fuse);
uint64_t sched_groups_grid(const SchedGroups& g);   // work groups launch_sched_groups runs

// H.v of a real-space problem (k_hv.hip).  pitch: elements from one row of
// x, y (and of the split and recurrence vectors) to the next; 0 means D_dn.
// A longer pitch (table path only) leaves columns D_dn..pitch-1 of every row
// as they are: zeros there stay zeros.
pdz_status launch_hv(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                     const int* skip = nullptr, unsigned passes = kPassDown | kPassUp,
                     const HvSplit* split = nullptr, uint64_t pitch = 0);
// H.v of any problem: momentum and parity sectors go to their kernels (every
// pass at once, no split form, no pitch), real-space problems to launch_hv.
pdz_status launch_hv_any(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                         const int* skip = nullptr, unsigned passes = kPassDown | kPassUp,
                         const HvSplit* split = nullptr, uint64_t pitch = 0);
bool hv_dot_counts(const pdz_problem_s* p, pdz_dtype dt, int* n_dn, int* n_up);   // false: no split path
size_t hv_dot_count_max(const pdz_problem_s* p, pdz_dtype dt);   // n_dn + n_up over every valid plan

}  // namespace pdz
