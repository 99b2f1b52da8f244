/*
 * A plain C client of libdsdp.so: no Python and no torch.  Device memory comes
 * from the HIP runtime (hipMalloc); everything else goes through the library's
 * C ABI (include/dsdp.h): receptor grid maps, then one dock on a stream of the
 * client's own.
 *
 * usage: c_client <request file> <result file>
 *
 * request (native byte order):
 *   int32  n_rec, n_types, n_atoms, n_frags, n_bonds, n_chains, n_steps, top_k
 *   uint64 seed
 *   float  box centre[3], size[3], spacing
 *   dsdp_atom receptor[n_rec]; int32 types[n_types]
 *   dsdp_atom ligand atoms[n_atoms]; int32 frag_start[n_frags + 1],
 *   frag_parent[n_frags], axis[2 n_frags], bonds[2 n_bonds]
 * result:
 *   int32 n_out; dsdp_pose poses[n_out]; int64 pose_evals, local_opts, accepted
 *
 * Exit status 0 on success; 1 after printing the library's or the runtime's
 * message.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "dsdp.h"

static FILE *in;

static void *take(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, in) != bytes) {
        fprintf(stderr, "c_client: short request file\n");
        exit(1);
    }
    return p;
}

static void check(dsdp_status st, const char *what)
{
    if (st != DSDP_OK) {
        fprintf(stderr, "c_client: %s failed (%d): %s\n", what, (int)st, dsdp_last_error());
        exit(1);
    }
}

static void check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        fprintf(stderr, "c_client: %s failed: %s\n", what, hipGetErrorString(e));
        exit(1);
    }
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: c_client <request file> <result file>\n");
        return 1;
    }
    in = fopen(argv[1], "rb");
    if (!in) {
        fprintf(stderr, "c_client: cannot open %s\n", argv[1]);
        return 1;
    }
    int32_t *h = take(8 * sizeof(int32_t));
    const int32_t n_rec = h[0], n_types = h[1], n_atoms = h[2], n_frags = h[3], n_bonds = h[4];
    const int32_t n_chains = h[5], n_steps = h[6], top_k = h[7];
    if (n_rec < 0 || n_types < 1 || n_atoms < 1 || n_frags < 1 || n_bonds < 0 || top_k < 1) {
        fprintf(stderr, "c_client: bad request header\n");
        return 1;
    }
    uint64_t *seed = take(sizeof(uint64_t));
    float *bf = take(7 * sizeof(float));
    dsdp_box box;
    for (int a = 0; a < 3; a++) {
        box.centre[a] = bf[a];
        box.size[a] = bf[3 + a];
    }
    box.spacing = bf[6];
    dsdp_atom *rec = take((size_t)n_rec * sizeof(dsdp_atom));
    int32_t *types = take((size_t)n_types * sizeof(int32_t));
    dsdp_atom *atoms = take((size_t)n_atoms * sizeof(dsdp_atom));
    int32_t *frag_start = take((size_t)(n_frags + 1) * sizeof(int32_t));
    int32_t *frag_parent = take((size_t)n_frags * sizeof(int32_t));
    int32_t *axis = take((size_t)2 * n_frags * sizeof(int32_t));
    int32_t *bonds = take((size_t)2 * n_bonds * sizeof(int32_t));
    fclose(in);

    hipStream_t stream;
    check_hip(hipStreamCreate(&stream), "hipStreamCreate");

    /* grid maps of the requested XS types */
    const size_t maps_bytes = dsdp_grids_bytes(&box, n_types);
    const size_t gws_bytes = dsdp_build_grids_workspace_bytes(n_rec, &box);
    if (maps_bytes == 0) {
        fprintf(stderr, "c_client: box has no nodes\n");
        return 1;
    }
    void *d_maps = NULL, *d_gws = NULL, *d_ws = NULL;
    check_hip(hipMalloc(&d_maps, maps_bytes), "hipMalloc maps");
    check_hip(hipMalloc(&d_gws, gws_bytes ? gws_bytes : 256), "hipMalloc grid workspace");
    dsdp_grids grids = NULL;
    check(dsdp_build_grids(rec, n_rec, &box, types, n_types, d_maps, maps_bytes, d_gws, gws_bytes, stream, &grids),
          "dsdp_build_grids");

    /* one dock with the default search constants */
    dsdp_ligand lig;
    lig.n_atoms = n_atoms;
    lig.atoms = atoms;
    lig.n_frags = n_frags;
    lig.frag_start = frag_start;
    lig.frag_parent = frag_parent;
    lig.axis = axis;
    lig.n_bonds = n_bonds;
    lig.bonds = bonds;
    dsdp_params prm;
    dsdp_params_default(&prm);
    const size_t ws_bytes = dsdp_dock_workspace_bytes(&lig, n_chains);
    if (ws_bytes == 0) check(DSDP_ERR_INVALID_ARG, "dsdp_dock_workspace_bytes");
    check_hip(hipMalloc(&d_ws, ws_bytes), "hipMalloc dock workspace");
    dsdp_pose *out = calloc((size_t)top_k, sizeof(dsdp_pose));
    int32_t n_out = 0;
    dsdp_dock_stats stats;
    check(dsdp_dock(grids, &lig, n_chains, n_steps, *seed, &prm, top_k, d_ws, ws_bytes, stream, out, NULL, &n_out,
                    NULL, &stats),
          "dsdp_dock");

    FILE *o = fopen(argv[2], "wb");
    if (!o) {
        fprintf(stderr, "c_client: cannot write %s\n", argv[2]);
        return 1;
    }
    const int64_t counts[3] = {stats.pose_evals, stats.local_opts, stats.accepted};
    if (fwrite(&n_out, sizeof n_out, 1, o) != 1 || fwrite(out, sizeof(dsdp_pose), (size_t)n_out, o) != (size_t)n_out ||
        fwrite(counts, sizeof counts, 1, o) != 1) {
        fprintf(stderr, "c_client: short write\n");
        return 1;
    }
    fclose(o);
    printf("c_client: %d poses, best e_total %.4f, %lld evaluations\n", (int)n_out, n_out ? out[0].e_total : 0.f,
           (long long)stats.pose_evals);

    dsdp_grids_release(grids);
    check_hip(hipFree(d_ws), "hipFree");
    check_hip(hipFree(d_gws), "hipFree");
    check_hip(hipFree(d_maps), "hipFree");
    check_hip(hipStreamDestroy(stream), "hipStreamDestroy");
    free(out);
    free(h); free(seed); free(bf); free(rec); free(types); free(atoms);
    free(frag_start); free(frag_parent); free(axis); free(bonds);
    return 0;
}
