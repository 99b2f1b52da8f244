// Host-side helpers of libdsdp shared by the C-ABI entry points and the serving
// scheduler.  Private to the library.
#pragma once

#include "../../include/dsdp.h"
#include "dsdp_internal.h"

#include <string>
#include <vector>

struct dsdp_grids_s {
    dsdp::GridView view;
    dsdp_box box;
    int types[dsdp::kNXS];
    int map_of_type[dsdp::kNXS];   // XS type -> map index or -1
    size_t bytes;
    std::vector<float4> site;      // adaptive search space (host copy)
    float site_r = 0.f;
};

namespace dsdp {
namespace host {

dsdp_status fail(dsdp_status code, const char *fmt, ...);
dsdp_status hip_fail(hipError_t e, const char *where);

#define HIP_TRY(expr, where)                                  \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return dsdp::host::hip_fail(e_, where); \
    } while (0)

constexpr size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
bool aligned256(const void *p);

// A ligand validated and packed into the blob the search kernels stage in LDS.
struct Prepared {
    LigHeader h;
    std::vector<uint32_t> blob;
    std::vector<int> map_index;   // per atom
};
// Where a prepared ligand will run: the caller's layout request
// (DSDP_INTRA_*), the chains of the launch and whether the launch mixes
// ligands.  With DSDP_INTRA_AUTO the layout follows choose_intra_form.
struct IntraCtx {
    int form = DSDP_INTRA_AUTO;
    long chains = 1;
    bool mixed = false;
};
IntraCtx intra_ctx(const dsdp_params *prm, long chains, bool mixed);
int choose_intra_form(int n_pairs, long chains, bool mixed);
dsdp_status prepare_ligand(const dsdp_ligand *lig, const int *map_of_type, Prepared &out, const IntraCtx &ctx);
// blob words of the larger of the two forms (workspace sizing without params); 0 on invalid input
size_t max_blob_words(const dsdp_ligand *lig);
dsdp_status check_params(const dsdp_params *p);
dsdp_status check_work(const dsdp_params *p, int32_t n_steps);
SearchParams to_search(const dsdp_params *p);
int device_cus();
size_t device_max_lds();
dsdp_status pick_waves(const dsdp_params *prm, const LigHeader &h, int n_chains, int &waves);
// One launch per kernel variant over the ligands that use it; each launch
// reserves its largest member's LDS for every workgroup.
struct LaunchGroup {
    int cls = 0, waves = 1;
    size_t lds = 0;
    long chains = 0;
    std::vector<int> members;   // indices into the caller's list
};
dsdp_status plan_groups(const dsdp_params *prm, const std::vector<const LigHeader *> &hdr,
                        const std::vector<long> &chains, std::vector<LaunchGroup> &out);

void fill_pose(const float *r, int nt, int chain, dsdp_pose &p);
void add_stats(const float *rec, long n, dsdp_dock_stats *stats);

}  // namespace host
}  // namespace dsdp
