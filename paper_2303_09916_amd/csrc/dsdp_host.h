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
    size_t bytes;
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
dsdp_status prepare_ligand(const dsdp_ligand *lig, const int *map_of_type, Prepared &out);
dsdp_status check_params(const dsdp_params *p);
SearchParams to_search(const dsdp_params *p);
int device_cus();
size_t device_max_lds();
dsdp_status pick_waves(const dsdp_params *prm, const LigHeader &h, int n_chains, int &waves);
void fill_pose(const float *r, int nt, int chain, dsdp_pose &p);
void add_stats(const float *rec, long n, dsdp_dock_stats *stats);

}  // namespace host
}  // namespace dsdp
