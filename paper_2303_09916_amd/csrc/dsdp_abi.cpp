// Host side of libdsdp.so: the C ABI declared in include/dsdp.h.
//
// Validates inputs, prepares the receptor (cell binning) and the ligand (torsion
// tree, intra-ligand pair list, packed blob) on the host -- the step in which
// the paper prepares the copies' initial data on the CPU (Section 2,
// parallelisation paragraph; Figure 4) -- uploads them, launches the gfx950
// kernels and turns the ranked chain results into output poses.
#include "../../include/dsdp.h"
#include "dsdp_internal.h"
#include "dsdp_host.h"
#include "tuner.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace dsdp;

namespace dsdp {
namespace host {

thread_local std::string g_error;

dsdp_status fail(dsdp_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

dsdp_status hip_fail(hipError_t e, const char *where)
{
    return fail(DSDP_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}


bool finite3(float a, float b, float c) { return std::isfinite(a) && std::isfinite(b) && std::isfinite(c); }

dsdp_status geometry(const dsdp_box *box, int n[3], double origin[3])
{
    if (!box) return fail(DSDP_ERR_INVALID_ARG, "box is NULL");
    if (!(std::isfinite(box->spacing) && box->spacing >= 0.05f && box->spacing <= 4.0f))
        return fail(DSDP_ERR_INVALID_ARG, "box spacing %g outside [0.05, 4] A", (double)box->spacing);
    for (int a = 0; a < 3; a++) {
        if (!std::isfinite(box->centre[a]) || !std::isfinite(box->size[a]))
            return fail(DSDP_ERR_INVALID_ARG, "box centre/size not finite");
        if (box->size[a] < box->spacing)
            return fail(DSDP_ERR_INVALID_ARG, "box size %g smaller than the spacing", (double)box->size[a]);
        const double nn = std::floor((double)box->size[a] / (double)box->spacing) + 1.0;
        if (nn > 2048) return fail(DSDP_ERR_UNSUPPORTED, "more than 2048 nodes per axis");
        n[a] = (int)nn;
        origin[a] = (double)box->centre[a] - 0.5 * (n[a] - 1) * (double)box->spacing;
    }
    if ((double)n[0] * n[1] * n[2] >= 2147483648.0)
        return fail(DSDP_ERR_UNSUPPORTED, "2^31 or more nodes per map");
    return DSDP_OK;
}

// cell binning geometry: the box grown by the cutoff, cell edge chosen so that a
// 8x8x4 node tile plus the cutoff spans at most 9 cells per axis
struct CellGeom {
    int cn[3];
    float clo[3];
    float cell;
    long ncell;
};
CellGeom cell_geometry(const int n[3], const double origin[3], double h)
{
    CellGeom c;
    c.cell = (float)std::max(4.0, (8.0 * h + 2.0 * kCutoff) / 9.0);
    c.ncell = 1;
    for (int a = 0; a < 3; a++) {
        const double lo = origin[a] - kCutoff, hi = origin[a] + (n[a] - 1) * h + kCutoff;
        c.clo[a] = (float)lo;
        c.cn[a] = (int)std::floor((hi - lo) / c.cell) + 1;
        c.ncell *= c.cn[a];
    }
    return c;
}

// ---------------------------------------------------------------- ligand preparation


dsdp_status validate_ligand(const dsdp_ligand *lig)
{
    if (!lig) return fail(DSDP_ERR_INVALID_ARG, "ligand is NULL");
    if (lig->n_atoms < 1) return fail(DSDP_ERR_INVALID_ARG, "ligand has %d atoms", lig->n_atoms);
    if (lig->n_atoms > kMaxAtoms) return fail(DSDP_ERR_UNSUPPORTED, "ligand has %d atoms (max %d)", lig->n_atoms, kMaxAtoms);
    if (lig->n_frags < 1) return fail(DSDP_ERR_INVALID_ARG, "ligand has %d fragments", lig->n_frags);
    if (lig->n_frags > kMaxFrags)
        return fail(DSDP_ERR_UNSUPPORTED, "ligand has %d torsions (max %d)", lig->n_frags - 1, kMaxTors);
    if (!lig->atoms || !lig->frag_start || !lig->frag_parent || (lig->n_frags > 1 && !lig->axis))
        return fail(DSDP_ERR_INVALID_ARG, "ligand array is NULL");
    if (lig->n_bonds < 0 || (lig->n_bonds > 0 && !lig->bonds)) return fail(DSDP_ERR_INVALID_ARG, "bad bond list");
    const int na = lig->n_atoms, nf = lig->n_frags;
    for (int i = 0; i < na; i++) {
        const dsdp_atom &a = lig->atoms[i];
        if (!finite3(a.x, a.y, a.z)) return fail(DSDP_ERR_INVALID_ARG, "ligand atom %d not finite", i);
        if (a.xs_type < 0 || a.xs_type >= kNXS) return fail(DSDP_ERR_INVALID_ARG, "ligand atom %d type %d", i, a.xs_type);
    }
    if (lig->frag_start[0] != 0 || lig->frag_start[nf] != na)
        return fail(DSDP_ERR_INVALID_ARG, "frag_start must run from 0 to n_atoms");
    for (int k = 0; k < nf; k++) {
        if (lig->frag_start[k + 1] <= lig->frag_start[k]) return fail(DSDP_ERR_INVALID_ARG, "fragment %d is empty", k);
        const int p = lig->frag_parent[k];
        if (k == 0 ? p != -1 : (p < 0 || p >= k))
            return fail(DSDP_ERR_INVALID_ARG, "fragment %d has parent %d (need -1 for the root, else < k)", k, p);
    }
    std::vector<int> frag_of(na);
    for (int k = 0; k < nf; k++)
        for (int i = lig->frag_start[k]; i < lig->frag_start[k + 1]; i++) frag_of[i] = k;
    std::vector<std::vector<int>> adj(na);
    for (int b = 0; b < lig->n_bonds; b++) {
        const int i = lig->bonds[2 * b], j = lig->bonds[2 * b + 1];
        if (i < 0 || i >= na || j < 0 || j >= na || i == j) return fail(DSDP_ERR_INVALID_ARG, "bond %d invalid", b);
        adj[i].push_back(j);
        adj[j].push_back(i);
    }
    for (int k = 1; k < nf; k++) {
        const int a = lig->axis[2 * k], b = lig->axis[2 * k + 1];
        if (a < 0 || a >= na || b < 0 || b >= na || frag_of[a] != lig->frag_parent[k] || frag_of[b] != k)
            return fail(DSDP_ERR_INVALID_ARG, "fragment %d axis (%d, %d) must join its parent to it", k, a, b);
        if (std::find(adj[a].begin(), adj[a].end(), b) == adj[a].end())
            return fail(DSDP_ERR_INVALID_ARG, "fragment %d axis (%d, %d) is not a bond", k, a, b);
        const float dx = lig->atoms[b].x - lig->atoms[a].x, dy = lig->atoms[b].y - lig->atoms[a].y,
                    dz = lig->atoms[b].z - lig->atoms[a].z;
        if (dx * dx + dy * dy + dz * dz < 1e-6f) return fail(DSDP_ERR_INVALID_ARG, "fragment %d axis has zero length", k);
    }
    return DSDP_OK;
}

// Layout of the intra-ligand term for a launch context (both give the same
// bits, so this only moves speed).  Measured on MI355X: pair lists are faster
// for one ligand's chains unless the ligand has many pairs and the chains fill
// the device; launches that mix ligands (batches, the scheduler) run faster
// with atom lists, whose smaller register and LDS footprint lets more
// workgroups share a compute unit.
int choose_intra_form(int n_pairs, long chains, bool mixed)
{
    if (mixed) return kFormAtoms;
    return (n_pairs > 600 && chains >= 2048) ? kFormAtoms : kFormPairs;
}

IntraCtx intra_ctx(const dsdp_params *prm, long chains, bool mixed)
{
    IntraCtx c;
    c.form = prm ? prm->intra_form : DSDP_INTRA_AUTO;
    c.chains = chains;
    c.mixed = mixed;
    return c;
}

// map_of_type == nullptr: map indices are left 0 (used only for sizing).
dsdp_status prepare_ligand(const dsdp_ligand *lig, const int *map_of_type, Prepared &out, const IntraCtx &ctx)
{
    const int form = ctx.form;
    dsdp_status st = validate_ligand(lig);
    if (st) return st;
    const int na = lig->n_atoms, nf = lig->n_frags;
    // atom slots: fragments in depth-first preorder (children by index), each
    // fragment's atoms in the caller's order; a subtree's atoms are then the
    // contiguous slots from its root fragment's first slot to its end
    std::vector<int> slot_atom, atom_slot(na), fs(nf), fe(nf), se(nf);
    {
        std::vector<std::vector<int>> kids(nf);
        for (int k = 1; k < nf; k++) kids[lig->frag_parent[k]].push_back(k);
        std::vector<int> stack{0}, order;
        while (!stack.empty()) {
            const int f = stack.back();
            stack.pop_back();
            order.push_back(f);
            for (auto it = kids[f].rbegin(); it != kids[f].rend(); ++it) stack.push_back(*it);
        }
        for (int f : order) {
            fs[f] = (int)slot_atom.size();
            for (int i = lig->frag_start[f]; i < lig->frag_start[f + 1]; i++) slot_atom.push_back(i);
            fe[f] = (int)slot_atom.size();
        }
        for (int v = 0; v < na; v++) atom_slot[slot_atom[v]] = v;
        // subtree ends: children follow their parent in the order, so a reverse
        // pass over it sees every child before its parent
        for (int f = 0; f < nf; f++) se[f] = fe[f];
        for (auto it = order.rbegin(); it != order.rend(); ++it)
            if (*it > 0) se[lig->frag_parent[*it]] = std::max(se[lig->frag_parent[*it]], se[*it]);
    }
    // from here on atoms are numbered by slot
    std::vector<int> frag_of(na);
    for (int k = 0; k < nf; k++)
        for (int v = fs[k]; v < fe[k]; v++) frag_of[v] = k;
    std::vector<double> ref(3 * na);
    std::vector<int> xs(na);
    for (int v = 0; v < na; v++) {
        const dsdp_atom &at = lig->atoms[slot_atom[v]];
        ref[3 * v] = at.x;
        ref[3 * v + 1] = at.y;
        ref[3 * v + 2] = at.z;
        xs[v] = at.xs_type;
    }
    // root centre and gyration radius
    double c0[3] = {0, 0, 0};
    const int n0 = fe[0];   // the root's atoms are slots [0, n0)
    for (int i = 0; i < n0; i++)
        for (int a = 0; a < 3; a++) c0[a] += ref[3 * i + a] / n0;
    double s2 = 0;
    for (int i = 0; i < na; i++)
        for (int a = 0; a < 3; a++) s2 += (ref[3 * i + a] - c0[a]) * (ref[3 * i + a] - c0[a]);
    const double rg = std::sqrt(s2 / na);
    auto frag_origin = [&](int k, double o[3]) {
        if (k == 0)
            for (int a = 0; a < 3; a++) o[a] = c0[a];
        else
            for (int a = 0; a < 3; a++) o[a] = ref[3 * atom_slot[lig->axis[2 * k + 1]] + a];
    };
    // bond-graph distances -> intra pairs (different fragments, > 3 bonds apart)
    std::vector<std::vector<int>> adj(na);
    for (int b = 0; b < lig->n_bonds; b++) {
        const int u = atom_slot[lig->bonds[2 * b]], v = atom_slot[lig->bonds[2 * b + 1]];
        adj[u].push_back(v);
        adj[v].push_back(u);
    }
    // pairs ordered by (j - i, i): 64 consecutive pairs (one wave-wide step of the
    // kernel) then touch distinct atoms
    std::vector<std::pair<int, int>> plist;
    for (int i = 0; i < na; i++) {
        std::vector<int> dist(na, 1 << 20), queue;
        dist[i] = 0;
        queue.push_back(i);
        for (size_t q = 0; q < queue.size(); q++)
            for (int v : adj[queue[q]])
                if (dist[v] > dist[queue[q]] + 1) {
                    dist[v] = dist[queue[q]] + 1;
                    queue.push_back(v);
                }
        for (int j = i + 1; j < na; j++)
            if (frag_of[i] != frag_of[j] && dist[j] > 3) plist.emplace_back(i, j);
    }
    std::stable_sort(plist.begin(), plist.end(), [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
        return (a.second - a.first) < (b.second - b.first);
    });
    std::vector<uint32_t> pairs;
    for (const auto &ij : plist) {
        const int i = ij.first, j = ij.second;
        pairs.push_back((uint32_t)i | ((uint32_t)j << 8) | (pair_flags(xs[i], xs[j]) << 16));
    }
    const int np = (int)pairs.size();
    // depth and subtree masks
    int max_depth = 0;
    std::vector<int> depth(nf, 0);
    for (int k = 1; k < nf; k++) {
        depth[k] = depth[lig->frag_parent[k]] + 1;
        max_depth = std::max(max_depth, depth[k]);
    }
    std::vector<uint32_t> sub(nf, 0);
    for (int m = 0; m < nf; m++)
        for (int x = m; x >= 0; x = lig->frag_parent[x]) sub[x] |= 1u << m;

    LigHeader h;
    std::memset(&h, 0, sizeof h);
    h.n_atoms = na;
    h.n_frags = nf;
    h.n_tors = nf - 1;
    h.n_pairs = np;
    h.max_depth = max_depth;
    h.rg = (float)rg;
    int w = kHeaderWords;
    auto take = [&](int words, int align) {
        w = (w + align - 1) / align * align;
        const int o = w;
        w += words;
        return o;
    };
    h.off_atom = take(4 * na, 4);
    h.off_frag_u = take(4 * nf, 4);
    h.off_frag_off = take(4 * nf, 4);
    h.off_atom_frag = take(na, 1);
    h.off_atom_ext = take(na, 1);
    h.off_frag_range = take(nf, 1);
    h.off_frag_anc = take(nf, 1);
    const int lpa = na <= 32 ? 2 : 1;
    h.lanes_per_atom = lpa;
    h.intra_form = form == DSDP_INTRA_PAIRS ? kFormPairs
                   : form == DSDP_INTRA_ATOMS ? kFormAtoms
                                              : choose_intra_form(np, ctx.chains, ctx.mixed);

    // per-lane lists of the chosen form.  Lane l serves atom l % 32 (every other
    // entry of the atom's list, from l / 32) when there are at most 32 atoms,
    // else atom l.
    //   pair lists: pair indices with a sign bit (set when the atom is the pair's
    //   second atom), padded with the zero slot n_pairs, 8 per 16-byte chunk;
    //   atom lists: partner bytes j | flags << 6, padded with kNbrNone, 4 per word
    std::vector<std::vector<uint16_t>> lane_list(64);
    std::vector<std::vector<uint8_t>> lane_nbr(64);
    size_t maxlen = 0;
    {
        std::vector<std::vector<uint16_t>> atom_list(na);
        std::vector<std::vector<uint8_t>> atom_nbr(na);
        for (int p = 0; p < np; p++) {
            const int i = pairs[p] & 255u, j = (pairs[p] >> 8) & 255u;
            const uint32_t fl = pairs[p] >> 16;
            atom_list[i].push_back((uint16_t)p);
            atom_list[j].push_back((uint16_t)(p | 0x8000));
            atom_nbr[i].push_back((uint8_t)(j | (fl << 6)));
            atom_nbr[j].push_back((uint8_t)(i | (fl << 6)));
        }
        for (int l = 0; l < 64; l++) {
            const int a = lpa == 2 ? (l & 31) : l, half = lpa == 2 ? (l >> 5) : 0;
            if (a >= na) continue;
            for (size_t e = half; e < atom_list[a].size(); e += lpa) {
                lane_list[l].push_back(atom_list[a][e]);
                lane_nbr[l].push_back(atom_nbr[a][e]);
            }
            maxlen = std::max(maxlen, lane_list[l].size());
        }
    }
    h.off_atom_rad = take(na, 1);
    if (h.intra_form == kFormPairs) {
        h.off_pair = take(np, 1);
        h.n_chunks = (int)((maxlen + 7) / 8);
        h.off_plist = take(h.n_chunks * 64 * 4, 4);
    } else {
        h.nbr_words = (int)((maxlen + 3) / 4);
        h.off_nbr = take(h.nbr_words * 64, 1);
    }
    h.total_words = (w + 3) / 4 * 4;

    std::vector<uint32_t> blob((size_t)h.total_words, 0u);
    std::memcpy(blob.data(), &h, sizeof h);
    auto fput = [&](int off, float v) { std::memcpy(&blob[(size_t)off], &v, 4); };
    out.map_index.assign(na, 0);
    for (int i = 0; i < na; i++) {
        double o[3];
        frag_origin(frag_of[i], o);
        const int t = xs[i];
        const int mi = map_of_type ? map_of_type[t] : 0;
        if (mi < 0) return fail(DSDP_ERR_INVALID_ARG, "no map for ligand atom %d of XS type %d", slot_atom[i], t);
        out.map_index[slot_atom[i]] = mi;
        for (int a = 0; a < 3; a++) fput(h.off_atom + 4 * i + a, (float)(ref[3 * i + a] - o[a]));
        blob[(size_t)h.off_atom + 4 * i + 3] = (uint32_t)mi;
        blob[(size_t)h.off_atom_frag + i] = (uint32_t)frag_of[i];
        blob[(size_t)h.off_atom_ext + i] = (uint32_t)slot_atom[i];
    }
    for (int k = 0; k < nf; k++) {
        if (k == 0) {
            for (int a = 0; a < 3; a++) fput(h.off_frag_u + a, 0.f);
            for (int a = 0; a < 3; a++) fput(h.off_frag_off + a, 0.f);
            blob[(size_t)h.off_frag_u + 3] = 0u;   // no parent, depth 0
        } else {
            const int ia = atom_slot[lig->axis[2 * k]], ib = atom_slot[lig->axis[2 * k + 1]];
            double u[3], nrm = 0, op[3];
            for (int a = 0; a < 3; a++) {
                u[a] = ref[3 * ib + a] - ref[3 * ia + a];
                nrm += u[a] * u[a];
            }
            nrm = std::sqrt(nrm);
            frag_origin(lig->frag_parent[k], op);
            for (int a = 0; a < 3; a++) {
                fput(h.off_frag_u + 4 * k + a, (float)(u[a] / nrm));
                fput(h.off_frag_off + 4 * k + a, (float)(ref[3 * ib + a] - op[a]));
            }
            blob[(size_t)h.off_frag_u + 4 * k + 3] = (uint32_t)(lig->frag_parent[k] + 1) | ((uint32_t)depth[k] << 16);
        }
        blob[(size_t)h.off_frag_off + 4 * k + 3] = sub[k];
    }
    for (int k = 0; k < nf; k++) {
        blob[(size_t)h.off_frag_range + k] = (uint32_t)fs[k] | ((uint32_t)fe[k] << 8) | ((uint32_t)se[k] << 16);
        uint32_t anc = 0;
        int b = 0;
        for (int m = k > 0 ? lig->frag_parent[k] : 0; m > 0 && b < 4; m = lig->frag_parent[m], b++)
            anc |= (uint32_t)m << (8 * b);
        blob[(size_t)h.off_frag_anc + k] = anc;
    }
    if (h.intra_form == kFormPairs) {
        for (int p = 0; p < np; p++) blob[(size_t)h.off_pair + p] = pairs[p];
        for (int c = 0; c < h.n_chunks; c++)
            for (int l = 0; l < 64; l++)
                for (int q = 0; q < 8; q++) {
                    const size_t e = (size_t)c * 8 + q;
                    const uint32_t v = e < lane_list[l].size() ? lane_list[l][e] : (uint32_t)np;
                    uint32_t &word = blob[(size_t)h.off_plist + ((size_t)c * 64 + l) * 4 + q / 2];
                    word |= (q & 1) ? (v << 16) : v;
                }
    } else {
        for (int m = 0; m < h.nbr_words; m++)
            for (int l = 0; l < 64; l++) {
                uint32_t word = 0;
                for (int b = 0; b < 4; b++) {
                    const size_t e = (size_t)m * 4 + b;
                    const uint32_t v = e < lane_nbr[l].size() ? lane_nbr[l][e] : kNbrNone;
                    word |= v << (8 * b);
                }
                blob[(size_t)h.off_nbr + (size_t)m * 64 + l] = word;
            }
    }
    for (int i = 0; i < na; i++) fput(h.off_atom_rad + i, xs_radius(xs[i]));
    out.h = h;
    out.blob.swap(blob);
    return DSDP_OK;
}

size_t max_blob_words(const dsdp_ligand *lig)
{
    Prepared a, b;
    if (prepare_ligand(lig, nullptr, a, IntraCtx{DSDP_INTRA_PAIRS}) || prepare_ligand(lig, nullptr, b, IntraCtx{DSDP_INTRA_ATOMS})) return 0;
    return (size_t)std::max(a.h.total_words, b.h.total_words);
}

SearchParams to_search(const dsdp_params *p)
{
    dsdp_params d;
    dsdp_params_default(&d);
    if (!p) p = &d;
    SearchParams s;
    s.temperature = p->temperature;
    s.wall_slope = p->wall_slope;
    s.rmsd_cluster = p->rmsd_cluster;
    s.trans_amp = p->trans_amp;
    s.bfgs_iters = p->bfgs_iters;
    s.ls_trials = p->ls_trials;
    s.ls_shrink = p->ls_shrink;
    s.armijo_c1 = p->armijo_c1;
    s.optimizer = p->optimizer;
    s.bb_iters = p->bb_iters;
    s.bb_step0 = p->bb_step0;
    s.bb_step_max = p->bb_step_max;
    s.ls_min_decrease = p->ls_min_decrease;
    return s;
}

dsdp_status check_params(const dsdp_params *p)
{
    if (!p) return DSDP_OK;
    if (p->struct_size != sizeof(dsdp_params)) return fail(DSDP_ERR_INVALID_ARG, "params.struct_size mismatch");
    if (!(p->temperature > 0) || !(p->wall_slope >= 0) || !(p->rmsd_cluster >= 0) || !(p->trans_amp >= 0) ||
        p->bfgs_iters < 0 || p->ls_trials < 1 || !(p->ls_shrink > 0 && p->ls_shrink < 1) || !(p->armijo_c1 >= 0) ||
        p->waves_per_chain < 0 || p->waves_per_chain > 4 || p->intra_form < DSDP_INTRA_AUTO ||
        p->intra_form > DSDP_INTRA_ATOMS || (p->optimizer != DSDP_OPT_BFGS && p->optimizer != DSDP_OPT_BB) ||
        p->bb_iters < 0 || !(p->bb_step0 > 0) || !(p->bb_step_max >= p->bb_step0) || !(p->ls_min_decrease >= 0) ||
        (p->tune != 0 && p->tune != 1))
        return fail(DSDP_ERR_INVALID_ARG, "search parameter out of range");
    return DSDP_OK;
}

// A chain counts its evaluations in 32 bits: n_steps local optimisations of at
// most 1 + bfgs_iters * ls_trials (BFGS) or 1 + bb_iters (Barzilai-Borwein)
// evaluations each must stay below 2^31.
dsdp_status check_work(const dsdp_params *p, int32_t n_steps)
{
    dsdp_params d;
    if (!p) {
        dsdp_params_default(&d);
        p = &d;
    }
    const double per_step = p->optimizer == DSDP_OPT_BB ? 1.0 + p->bb_iters : 1.0 + (double)p->bfgs_iters * p->ls_trials;
    if ((double)n_steps * per_step >= 2147483647.0)
        return fail(DSDP_ERR_UNSUPPORTED, "n_steps %d x %.0f evaluations per step: a chain's count would exceed 2^31",
                    n_steps, per_step);
    return DSDP_OK;
}

// Workspace layout of the search calls.  The host-written sections (blob arena,
// tasks, grid views, ranking segments) come first and are uploaded in one copy.
struct SearchWs {
    size_t arena, tasks, grids, site, segs, host_end, state, records, xyz, sel, total;
};
SearchWs search_ws(size_t arena_words, long n_slots, int n_grids, int n_segs)
{
    SearchWs w;
    size_t o = 0;
    w.arena = o; o += align256(arena_words * 4);
    w.tasks = o; o += align256((size_t)n_slots * sizeof(ChainTask));
    w.grids = o; o += align256((size_t)n_grids * sizeof(GridView));
    w.site = o; o += align256((size_t)kMaxSite * sizeof(float4));
    w.segs = o; o += align256((size_t)n_segs * sizeof(RankSeg));
    w.host_end = o;
    w.state = o; o += align256((size_t)n_slots * kStWords * 4);
    w.records = o; o += align256((size_t)n_slots * kRecWords * 4);
    w.xyz = o; o += align256((size_t)n_slots * kXyzStride * 16);
    w.sel = o; o += align256((size_t)(n_slots + n_segs) * 4);
    w.total = o;
    return w;
}
SearchWs search_ws(const LigHeader &h, int n) { return search_ws((size_t)h.total_words, n, 1, 1); }

// The grids' device view for a workspace whose site section (at ws + w.site)
// receives the search-space points; `host` (nullable) is the host image of the
// workspace's host-written part, else the points are copied on `stream`.
dsdp_status device_view(const dsdp_grids_s *g, char *ws, const SearchWs &w, unsigned char *host, hipStream_t stream,
                        GridView &view)
{
    view = g->view;
    view.n_site = (int)g->site.size();
    view.site_r = g->site_r;
    view.site = view.n_site ? (const float4 *)(ws + w.site) : nullptr;
    if (!view.n_site) return DSDP_OK;
    const size_t bytes = g->site.size() * sizeof(float4);
    if (host) {
        std::memcpy(host + w.site, g->site.data(), bytes);
        return DSDP_OK;
    }
    HIP_TRY(hipMemcpyAsync(ws + w.site, g->site.data(), bytes, hipMemcpyHostToDevice, stream), "site upload");
    HIP_TRY(hipStreamSynchronize(stream), "site upload");
    return DSDP_OK;
}

dsdp_status upload_blob(const Prepared &pl, char *d_ws, hipStream_t stream)
{
    HIP_TRY(hipMemcpyAsync(d_ws, pl.blob.data(), pl.blob.size() * 4, hipMemcpyHostToDevice, stream), "ligand upload");
    // the host blob is freed when the caller returns: wait for the copy
    HIP_TRY(hipStreamSynchronize(stream), "ligand upload");
    return DSDP_OK;
}

// Host image of the first workspace sections, uploaded in one copy.
struct HostImage {
    std::vector<unsigned char> bytes;
    explicit HostImage(size_t n) : bytes(n, 0) {}
    template <typename T> T *at(size_t off) { return reinterpret_cast<T *>(bytes.data() + off); }
};

bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

// Compute units of the current device (cached per device).
int device_cus()
{
    static thread_local int dev_cached = -1, cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev != dev_cached) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus = v;
        dev_cached = dev;
    }
    return cus;
}

// LDS bytes a workgroup may use on the current device.
size_t device_max_lds()
{
    static thread_local int dev_cached = -1;
    static thread_local size_t bytes = 65536;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (dev != dev_cached) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        bytes = (size_t)v;
        dev_cached = dev;
    }
    return bytes;
}

// Waves per chain: the caller's choice, else about 8 waves per compute unit
// (measured on MI355X with a 32-atom ligand: 4 waves per chain at 384 chains,
// 2 at 1024, 1 at 4096 chains); every choice gives the same results.  Reduced
// until the workgroup's LDS fits the device's limit.
dsdp_status pick_waves(const dsdp_params *prm, const LigHeader &h, int n_chains, int &waves)
{
    int w = (prm && prm->waves_per_chain > 0) ? prm->waves_per_chain : 0;
    // Barzilai-Borwein evaluates one point per iteration: with atom lists one
    // wave does all of it (more would idle); pair lists spread its pairs over
    // the waves
    if (w == 0 && prm && prm->optimizer == DSDP_OPT_BB && h.intra_form != kFormPairs) w = 1;
    if (w == 0) {
        const long slots = 8L * device_cus();
        w = (int)std::max(1L, std::min(4L, slots / std::max(1, n_chains)));
    }
    const size_t cap = device_max_lds();
    while (w > 1 && search_lds_bytes(h, w) > cap) w--;
    if (search_lds_bytes(h, w) > cap)
        return fail(DSDP_ERR_UNSUPPORTED, "ligand needs %zu bytes of LDS per chain", search_lds_bytes(h, 1));
    waves = w;
    return DSDP_OK;
}

// HIP events released on every return path
struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    hipError_t create()
    {
        for (auto &x : e) {
            hipError_t r = hipEventCreate(&x);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    ~Events()
    {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

dsdp_status plan_groups(const dsdp_params *prm, const std::vector<const LigHeader *> &hdr,
                        const std::vector<long> &chains, std::vector<LaunchGroup> &out)
{
    out.clear();
    const int n = (int)hdr.size();
    std::vector<int> idx(n);
    std::vector<size_t> lds1(n);
    for (int i = 0; i < n; i++) {
        idx[i] = i;
        lds1[i] = search_lds_bytes(*hdr[i], 1);
    }
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        const int ca = search_class(*hdr[a]), cb = search_class(*hdr[b]);
        return ca != cb ? ca < cb : lds1[a] < lds1[b];
    });
    for (int k = 0; k < n;) {
        LaunchGroup g;
        g.cls = search_class(*hdr[idx[k]]);
        int worst = idx[k];
        while (k < n && search_class(*hdr[idx[k]]) == g.cls) {
            g.members.push_back(idx[k]);
            g.chains += chains[idx[k]];
            worst = idx[k];   // sorted by LDS: the last member needs the most
            k++;
        }
        // waves per chain from the group's chain count (groups are launched one
        // after another), then lowered until the largest member fits
        dsdp_status st = pick_waves(prm, *hdr[worst], (int)std::min<long>(g.chains, 1L << 30), g.waves);
        if (st) return st;
        for (;;) {
            g.lds = search_lds_bytes(*hdr[worst], g.waves);
            if (g.lds <= device_max_lds() || g.waves == 1) break;
            g.waves--;
        }
        if (g.lds > device_max_lds()) return fail(DSDP_ERR_UNSUPPORTED, "a ligand needs %zu bytes of LDS", g.lds);
        out.push_back(std::move(g));
    }
    return DSDP_OK;
}

void fill_pose(const float *r, int nt, int chain, dsdp_pose &p)
{
    std::memset(&p, 0, sizeof p);
    for (int a = 0; a < 3; a++) p.pos[a] = r[kRecPose + a];
    for (int a = 0; a < 4; a++) p.quat[a] = r[kRecPose + 3 + a];
    for (int k = 0; k < nt; k++) p.tors[k] = r[kRecPose + 7 + k];
    p.e_total = r[kRecE];
    p.e_inter = r[kRecE + 1];
    p.e_intra = r[kRecE + 2];
    p.e_wall = r[kRecE + 3];
    p.score = p.e_inter / (1.0f + kWRot * (float)nt);
    p.chain = chain;
}

void add_stats(const float *rec, long n, dsdp_dock_stats *stats)
{
    for (long c = 0; c < n; c++) {
        const int *ri = reinterpret_cast<const int *>(rec + c * kRecWords);
        stats->pose_evals += ri[kRecEvals];
        stats->accepted += ri[kRecAccepted];
        stats->local_opts += ri[kRecLocalOpts];
        if (!std::isfinite(rec[c * kRecWords + kRecE])) stats->n_nonfinite++;
    }
}

}  // namespace host
}  // namespace dsdp

using namespace dsdp::host;

extern "C" {

const char *dsdp_last_error(void) { return g_error.c_str(); }

const char *dsdp_version(void) { return "dsdp-mi355x 0.1 (gfx950)"; }

void dsdp_params_default(dsdp_params *p)
{
    if (!p) return;
    p->struct_size = sizeof(dsdp_params);
    p->temperature = 1.2f;
    p->wall_slope = 10.0f;
    p->rmsd_cluster = 1.0f;
    p->trans_amp = 2.0f;
    p->bfgs_iters = 20;
    p->ls_trials = 10;
    p->ls_shrink = 0.1f;
    p->armijo_c1 = 1e-4f;
    p->waves_per_chain = 0;
    p->intra_form = DSDP_INTRA_AUTO;
    p->optimizer = DSDP_OPT_BFGS;
    p->bb_iters = 100;
    p->bb_step0 = 1e-2f;
    p->bb_step_max = 1.0f;
    p->ls_min_decrease = 1e-4f;
    p->tune = 1;
}

dsdp_status dsdp_grid_dims(const dsdp_box *box, int32_t *n, float *origin)
{
    int nn[3];
    double o[3];
    dsdp_status st = geometry(box, nn, o);
    if (st) return st;
    for (int a = 0; a < 3; a++) {
        if (n) n[a] = nn[a];
        if (origin) origin[a] = (float)o[a];
    }
    return DSDP_OK;
}

size_t dsdp_grids_bytes(const dsdp_box *box, int32_t n_types)
{
    int n[3];
    double o[3];
    if (n_types < 1 || n_types > kNXS || geometry(box, n, o)) return 0;
    return (size_t)n[0] * n[1] * n[2] * (size_t)n_types * 16;
}

size_t dsdp_build_grids_workspace_bytes(int32_t n_rec, const dsdp_box *box)
{
    int n[3];
    double o[3];
    if (n_rec < 0 || geometry(box, n, o)) return 0;
    const CellGeom c = cell_geometry(n, o, box->spacing);
    return align256((size_t)std::max(n_rec, 1) * 16) + align256((size_t)(c.ncell + 1) * 4);
}

dsdp_status dsdp_build_grids(const dsdp_atom *rec, int32_t n_rec, const dsdp_box *box, const int32_t *types,
                             int32_t n_types, void *d_maps, size_t maps_bytes, void *d_ws, size_t ws_bytes,
                             void *stream, dsdp_grids *out)
{
    if (!out) return fail(DSDP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n[3];
    double origin[3];
    dsdp_status st = geometry(box, n, origin);
    if (st) return st;
    if (n_rec < 0 || (n_rec > 0 && !rec)) return fail(DSDP_ERR_INVALID_ARG, "bad receptor array");
    int tl[kNXS];
    if (!types) {
        n_types = kNXS;
        for (int t = 0; t < kNXS; t++) tl[t] = t;
    } else {
        if (n_types < 1 || n_types > kNXS) return fail(DSDP_ERR_INVALID_ARG, "n_types %d outside 1..17", n_types);
        for (int t = 0; t < n_types; t++) {
            if (types[t] < 0 || types[t] >= kNXS) return fail(DSDP_ERR_INVALID_ARG, "map type %d invalid", types[t]);
            for (int u = 0; u < t; u++)
                if (types[u] == types[t]) return fail(DSDP_ERR_INVALID_ARG, "map type %d repeated", types[t]);
            tl[t] = types[t];
        }
    }
    for (int j = 0; j < n_rec; j++) {
        if (!finite3(rec[j].x, rec[j].y, rec[j].z)) return fail(DSDP_ERR_INVALID_ARG, "receptor atom %d not finite", j);
        if (rec[j].xs_type < 0 || rec[j].xs_type >= kNXS)
            return fail(DSDP_ERR_INVALID_ARG, "receptor atom %d type %d", j, rec[j].xs_type);
    }
    const size_t need = dsdp_grids_bytes(box, n_types);
    if (!d_maps || maps_bytes < need)
        return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "maps need %zu bytes, got %zu", need, maps_bytes);
    const size_t wneed = dsdp_build_grids_workspace_bytes(n_rec, box);
    if (!d_ws || ws_bytes < wneed)
        return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes, got %zu", wneed, ws_bytes);
    if (!aligned256(d_maps) || !aligned256(d_ws)) return fail(DSDP_ERR_INVALID_ARG, "device buffers must be 256-byte aligned");

    // receptor prep: keep atoms within the cutoff of the box, counting sort by cell
    const CellGeom cg = cell_geometry(n, origin, box->spacing);
    std::vector<int> key;
    std::vector<int> keep;
    key.reserve(n_rec);
    keep.reserve(n_rec);
    for (int j = 0; j < n_rec; j++) {
        const double p[3] = {rec[j].x, rec[j].y, rec[j].z};
        int c[3];
        bool in = true;
        for (int a = 0; a < 3; a++) {
            const double lo = origin[a] - kCutoff, hi = origin[a] + (n[a] - 1) * (double)box->spacing + kCutoff;
            if (p[a] < lo || p[a] > hi) in = false;
            c[a] = std::min(cg.cn[a] - 1, std::max(0, (int)std::floor((p[a] - cg.clo[a]) / cg.cell)));
        }
        if (!in) continue;
        keep.push_back(j);
        key.push_back((c[2] * cg.cn[1] + c[1]) * cg.cn[0] + c[0]);
    }
    std::vector<int> start((size_t)cg.ncell + 1, 0);
    for (int k : key) start[(size_t)k + 1]++;
    for (long c = 0; c < cg.ncell; c++) start[(size_t)c + 1] += start[(size_t)c];
    std::vector<int> fill(start.begin(), start.end() - 1);
    std::vector<float4> sorted(std::max<size_t>(keep.size(), 1));
    for (size_t q = 0; q < keep.size(); q++) {
        const dsdp_atom &a = rec[keep[q]];
        float4 v;
        v.x = a.x; v.y = a.y; v.z = a.z;
        std::memcpy(&v.w, &a.xs_type, 4);
        sorted[(size_t)fill[(size_t)key[q]]++] = v;
    }
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    float4 *d_atoms = (float4 *)ws;
    int *d_start = (int *)(ws + align256((size_t)std::max(n_rec, 1) * 16));
    HIP_TRY(hipMemcpyAsync(d_atoms, sorted.data(), keep.size() * sizeof(float4), hipMemcpyHostToDevice, s), "receptor upload");
    HIP_TRY(hipMemcpyAsync(d_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice, s), "cell upload");
    HIP_TRY(hipStreamSynchronize(s), "receptor upload");

    dsdp_grids g = new dsdp_grids_s();
    g->box = *box;
    g->bytes = need;
    g->view.maps = (const float4 *)d_maps;
    for (int a = 0; a < 3; a++) {
        g->view.n[a] = n[a];
        g->view.origin[a] = (float)origin[a];
    }
    g->view.h = box->spacing;
    g->view.inv_h = 1.0f / box->spacing;
    g->view.T = n_types;
    g->view.site = nullptr;
    g->view.n_site = 0;
    g->view.site_r = 0.f;
    for (int t = 0; t < kNXS; t++) g->map_of_type[t] = -1;
    for (int t = 0; t < n_types; t++) {
        g->map_of_type[tl[t]] = t;
        g->types[t] = tl[t];
    }
    hipError_t e = launch_grid_build(d_atoms, d_start, cg.cn, cg.clo, cg.cell, g->view, tl, (float4 *)d_maps, s);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "grid build launch");
    }
    *out = g;
    return DSDP_OK;
}

void dsdp_grids_release(dsdp_grids g) { delete g; }

size_t dsdp_gather_probe_workspace_bytes(int32_t blocks)
{
    return blocks < 1 ? 0 : align256((size_t)blocks * 256 * 4);
}

dsdp_status dsdp_gather_probe(dsdp_grids g, int32_t blocks, int32_t rounds, uint64_t seed, void *d_ws,
                              size_t ws_bytes, void *stream, double *bytes_per_s)
{
    if (!g || !bytes_per_s) return fail(DSDP_ERR_INVALID_ARG, "grids or result is NULL");
    if (blocks < 1 || blocks > (1 << 20) || rounds < 1 || rounds > (1 << 16))
        return fail(DSDP_ERR_INVALID_ARG, "blocks must be in [1, 2^20] and rounds in [1, 2^16]");
    const size_t need = dsdp_gather_probe_workspace_bytes(blocks);
    if (!d_ws || ws_bytes < need) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    Events ev;
    HIP_TRY(ev.create(), "event");
    HIP_TRY(launch_gather_probe(g->view, blocks, 1, (uint32_t)seed, (float *)d_ws, s), "probe launch");
    HIP_TRY(hipEventRecord(ev.e[0], s), "event");
    HIP_TRY(launch_gather_probe(g->view, blocks, rounds, (uint32_t)(seed >> 32) ^ 0x5bd1e995u, (float *)d_ws, s),
            "probe launch");
    HIP_TRY(hipEventRecord(ev.e[1], s), "event");
    HIP_TRY(hipEventSynchronize(ev.e[1]), "probe");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]), "event");
    *bytes_per_s = (double)blocks * 256.0 * rounds * 128.0 / (ms * 1e-3);
    return DSDP_OK;
}

dsdp_status dsdp_valu_probe(int32_t blocks, int32_t iters, void *d_ws, size_t ws_bytes, void *stream,
                            double *flops_per_s)
{
    if (!flops_per_s) return fail(DSDP_ERR_INVALID_ARG, "result is NULL");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 20))
        return fail(DSDP_ERR_INVALID_ARG, "blocks and iters must be in [1, 2^20]");
    const size_t need = dsdp_gather_probe_workspace_bytes(blocks);
    if (!d_ws || ws_bytes < need) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", need);
    hipStream_t s = (hipStream_t)stream;
    Events ev;
    HIP_TRY(ev.create(), "event");
    HIP_TRY(launch_valu_probe(blocks, 1, 1.f, (float *)d_ws, s), "probe launch");
    HIP_TRY(hipEventRecord(ev.e[0], s), "event");
    HIP_TRY(launch_valu_probe(blocks, iters, 2.f, (float *)d_ws, s), "probe launch");
    HIP_TRY(hipEventRecord(ev.e[1], s), "event");
    HIP_TRY(hipEventSynchronize(ev.e[1]), "probe");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]), "event");
    *flops_per_s = 2.0 * 8.0 * (double)iters * (double)blocks * 256.0 / (ms * 1e-3);
    return DSDP_OK;
}

size_t dsdp_site_points_workspace_bytes(int32_t top_n)
{
    if (top_n < 1 || top_n > kMaxSitePoints) return 0;
    return align256((size_t)top_n * 8);
}

dsdp_status dsdp_site_points(const float *d_scores, const int32_t *dims, const float *origin, float spacing,
                             int32_t top_n, float link_dist, void *d_ws, size_t ws_bytes, void *stream,
                             float *points, int32_t *labels, int32_t *n_out, float *centre)
{
    if (!d_scores || !dims || !origin || !points || !labels || !n_out)
        return fail(DSDP_ERR_INVALID_ARG, "scores, dims, origin or an output is NULL");
    if (top_n < 1 || top_n > kMaxSitePoints) return fail(DSDP_ERR_INVALID_ARG, "top_n %d outside 1..%d", top_n, kMaxSitePoints);
    if (!(spacing > 0.f) || !std::isfinite(spacing)) return fail(DSDP_ERR_INVALID_ARG, "spacing must be positive");
    long n = 1;
    for (int a = 0; a < 3; a++) {
        if (dims[a] < 1) return fail(DSDP_ERR_INVALID_ARG, "dims must be positive");
        n *= dims[a];
    }
    if (n > (1L << 26)) return fail(DSDP_ERR_UNSUPPORTED, "more than 2^26 voxels");
    const size_t need = dsdp_site_points_workspace_bytes(top_n);
    if (!d_ws || ws_bytes < need) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", need);
    const int k = (int)std::min<long>(top_n, n);
    const double link = link_dist > 0.f ? (double)link_dist : std::sqrt(3.0) * spacing;
    const int lim = (int)std::floor(link * link / ((double)spacing * spacing) + 1e-9);
    hipStream_t s = (hipStream_t)stream;
    int *d_index = (int *)d_ws, *d_label = d_index + top_n;
    const int dm[3] = {dims[0], dims[1], dims[2]};
    HIP_TRY(launch_site_extract(d_scores, dm, k, lim, d_index, d_label, s), "site extraction launch");
    std::vector<int> h((size_t)2 * top_n);
    HIP_TRY(hipMemcpyAsync(h.data(), d_index, h.size() * 4, hipMemcpyDeviceToHost, s), "site copy");
    HIP_TRY(hipStreamSynchronize(s), "site extraction");
    for (int a = 0; a < k; a++) {
        const int idx = h[(size_t)a];
        const int ijk[3] = {idx % dims[0], (idx / dims[0]) % dims[1], idx / (dims[0] * dims[1])};
        for (int c = 0; c < 3; c++) points[3 * a + c] = origin[c] + (float)ijk[c] * spacing;
        labels[a] = h[(size_t)top_n + a];
    }
    if (centre)
        for (int c = 0; c < 3; c++) centre[c] = points[c];
    *n_out = k;
    return DSDP_OK;
}

dsdp_status dsdp_grids_set_site(dsdp_grids g, const float *points, int32_t n_points, float radius)
{
    if (!g) return fail(DSDP_ERR_INVALID_ARG, "grids handle is NULL");
    if (n_points < 0 || n_points > kMaxSite) return fail(DSDP_ERR_INVALID_ARG, "n_points %d outside 0..%d", n_points, kMaxSite);
    if (n_points > 0 && (!points || !(radius > 0.f) || !std::isfinite(radius)))
        return fail(DSDP_ERR_INVALID_ARG, "site points missing or radius not positive");
    std::vector<float4> site((size_t)n_points);
    for (int i = 0; i < n_points; i++) {
        const float x = points[3 * i], y = points[3 * i + 1], z = points[3 * i + 2];
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
            return fail(DSDP_ERR_INVALID_ARG, "site point %d is not finite", i);
        site[(size_t)i] = make_float4(x, y, z, 0.f);
    }
    g->site.swap(site);
    g->site_r = n_points ? radius : 0.f;
    return DSDP_OK;
}

dsdp_status dsdp_ligand_info(const dsdp_ligand *lig, int32_t *n_pairs, int32_t *tree_depth)
{
    Prepared pl;
    dsdp_status st = prepare_ligand(lig, nullptr, pl, IntraCtx{});
    if (st) return st;
    if (n_pairs) *n_pairs = pl.h.n_pairs;
    if (tree_depth) *tree_depth = pl.h.max_depth;
    return DSDP_OK;
}

size_t dsdp_dock_workspace_bytes(const dsdp_ligand *lig, int32_t n_chains)
{
    const size_t words = max_blob_words(lig);
    if (n_chains < 1 || words == 0) return 0;
    return search_ws(words, n_chains, 1, 1).total;
}

dsdp_status dsdp_eval_poses(dsdp_grids g, const dsdp_ligand *lig, const float *d_poses, int32_t n_poses,
                            const dsdp_params *prm, float *d_energy, float *d_grad, float *d_xyz, void *d_ws,
                            size_t ws_bytes, void *stream)
{
    if (!g) return fail(DSDP_ERR_INVALID_ARG, "grids handle is NULL");
    if (n_poses < 0) return fail(DSDP_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses > 0 && (!d_poses || !d_energy || !d_grad)) return fail(DSDP_ERR_INVALID_ARG, "device array is NULL");
    dsdp_status st = check_params(prm);
    if (st) return st;
    Prepared pl;
    st = prepare_ligand(lig, g->map_of_type, pl, intra_ctx(prm, n_poses, false));
    if (st) return st;
    const SearchWs w = search_ws(pl.h, std::max(n_poses, 1));
    if (!d_ws || ws_bytes < w.total) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
    if (!aligned256(d_ws)) return fail(DSDP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (n_poses == 0) return DSDP_OK;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    st = upload_blob(pl, ws + w.arena, s);
    if (st) return st;
    GridView view;
    st = device_view(g, ws, w, nullptr, s, view);
    if (st) return st;
    HIP_TRY(launch_eval((const uint32_t *)(ws + w.arena), pl.h.total_words, pl.h, view, to_search(prm), d_poses,
                        n_poses, d_energy, d_grad, d_xyz, s),
            "eval launch");
    return DSDP_OK;
}

dsdp_status dsdp_local_opt(dsdp_grids g, const dsdp_ligand *lig, const float *d_poses_in, int32_t n_poses,
                           const dsdp_params *prm, float *d_poses_out, float *d_energy, int32_t *d_evals,
                           void *d_ws, size_t ws_bytes, void *stream)
{
    if (!g) return fail(DSDP_ERR_INVALID_ARG, "grids handle is NULL");
    if (n_poses < 0) return fail(DSDP_ERR_INVALID_ARG, "n_poses < 0");
    if (n_poses > 0 && (!d_poses_in || !d_poses_out || !d_energy))
        return fail(DSDP_ERR_INVALID_ARG, "device array is NULL");
    dsdp_status st = check_params(prm);
    if (st) return st;
    Prepared pl;
    st = prepare_ligand(lig, g->map_of_type, pl, intra_ctx(prm, n_poses, false));
    if (st) return st;
    const SearchWs w = search_ws(pl.h, std::max(n_poses, 1));
    if (!d_ws || ws_bytes < w.total) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
    if (!aligned256(d_ws)) return fail(DSDP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (n_poses == 0) return DSDP_OK;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    st = upload_blob(pl, ws + w.arena, s);
    if (st) return st;
    int waves = 1;
    st = pick_waves(prm, pl.h, n_poses, waves);
    if (st) return st;
    GridView view;
    st = device_view(g, ws, w, nullptr, s, view);
    if (st) return st;
    HIP_TRY(launch_local_opt((const uint32_t *)(ws + w.arena), pl.h.total_words, pl.h, view, to_search(prm), waves,
                             d_poses_in, n_poses, d_poses_out, d_energy, d_evals, s),
            "local-opt launch");
    return DSDP_OK;
}

}  // extern "C"

namespace {

Tuner &tuner()
{
    static Tuner t;
    return t;
}

constexpr int kTrialSteps = 4;   // timed MC steps of a tuner trial (every chain of the request)

// The workspace's host-written part for one dock (blob, chain tasks from fresh
// starts, grid view, ranking segment), uploaded on s.
dsdp_status upload_dock(const dsdp_grids_s *g, const Prepared &pl, const SearchWs &w, int n_chains, int n_steps,
                        uint64_t seed, int top_k, char *ws, hipStream_t s)
{
    HostImage img(w.host_end);
    std::memcpy(img.at<uint32_t>(w.arena), pl.blob.data(), pl.blob.size() * 4);
    ChainTask *tasks = img.at<ChainTask>(w.tasks);
    for (int c = 0; c < n_chains; c++) {
        ChainTask &t = tasks[c];
        t.blob_off = 0;
        t.blob_words = (uint32_t)pl.h.total_words;
        t.chain = (uint32_t)c;
        t.n_steps = n_steps;
        t.seed_lo = (uint32_t)seed;
        t.seed_hi = (uint32_t)(seed >> 32);
        t.grid = 0;
        t.slot = c;
        t.fresh = 1;
    }
    GridView view;
    dsdp_status st = device_view(g, ws, w, img.bytes.data(), s, view);
    if (st) return st;
    *img.at<GridView>(w.grids) = view;
    RankSeg *seg = img.at<RankSeg>(w.segs);
    seg->slot0 = 0;
    seg->n_chains = n_chains;
    seg->n_atoms = pl.h.n_atoms;
    seg->top_k = top_k;
    seg->sel_off = 0;
    HIP_TRY(hipMemcpyAsync(ws, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice, s), "task upload");
    HIP_TRY(hipStreamSynchronize(s), "task upload");
    return DSDP_OK;
}

// The tuned layout and waves of a dock: the cached pick for the request's
// make-up (optimiser, ligand shape, chains), else each candidate timed on a
// trial of the request itself (every chain, one untimed step from fresh starts
// and then the next kTrialSteps steps timed, on the caller's workspace) and the
// fastest cached.  With lookup_only nothing is measured (waves stays 0 without a
// cached pick).  `use` is pl or alt (the other layout, prepared here).
dsdp_status tune_dock(const dsdp_grids_s *g, const dsdp_ligand *lig, const dsdp_params *prm, const Prepared &pl,
                      Prepared &alt, int n_chains, uint64_t seed, const SearchParams &sp, char *ws, size_t ws_bytes,
                      hipStream_t s, bool lookup_only, const Prepared *&use, int &waves)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "device");
    const int kind = prm->optimizer == DSDP_OPT_BB ? kTuneDockBb : kTuneDockBfgs;
    const TuneKey key = tune_key(dev, n_chains, {shape_bucket(pl.h.n_atoms, pl.h.n_pairs, 6 + pl.h.n_tors)}, kind);
    const int pl_form = pl.h.intra_form == kFormPairs ? DSDP_INTRA_PAIRS : DSDP_INTRA_ATOMS;
    bool have_alt = false;
    dsdp_status mst = DSDP_OK;
    auto layout = [&](int form) -> const Prepared * {
        if (form == pl_form) return &pl;
        if (!have_alt) {
            if ((mst = prepare_ligand(lig, g->map_of_type, alt, IntraCtx{form}))) return nullptr;
            have_alt = true;
        }
        return &alt;
    };
    int pick = -1;
    if (lookup_only) {
        if (!tuner().find(key, pick)) return DSDP_OK;
    } else {
        auto measure = [&](int c) -> float {
            const DockCandidate dc = dock_candidate(c);
            const Prepared *P = mst ? nullptr : layout(dc.form);
            if (!P) return -1.f;
            const size_t lds = search_lds_bytes(P->h, dc.waves);
            const SearchWs w = search_ws(P->h, n_chains);
            if (lds > device_max_lds() || w.total > ws_bytes) return -1.f;
            // trial chains run 1 + kTrialSteps steps whatever the request's length,
            // so that requests of any length share the cached pick
            if ((mst = upload_dock(g, *P, w, n_chains, 1 + kTrialSteps, seed, 0, ws, s))) return -1.f;
            Events ev;
            float ms = -1.f;
            auto tick = [&](int steps, int init) {
                return launch_tick(search_class(P->h), dc.waves, lds, (const uint32_t *)(ws + w.arena),
                                   (const ChainTask *)(ws + w.tasks), n_chains, (const GridView *)(ws + w.grids), sp,
                                   steps, init, (float *)(ws + w.state), (float *)(ws + w.records),
                                   (float4 *)(ws + w.xyz), s);
            };
            const bool ok = ev.create() == hipSuccess && tick(1, 1) == hipSuccess &&
                            hipEventRecord(ev.e[0], s) == hipSuccess && tick(kTrialSteps, 0) == hipSuccess &&
                            hipEventRecord(ev.e[1], s) == hipSuccess && hipEventSynchronize(ev.e[1]) == hipSuccess &&
                            hipEventElapsedTime(&ms, ev.e[0], ev.e[1]) == hipSuccess;
            if (!ok) mst = fail(DSDP_ERR_DEVICE, "dock tuner trial: %s", hipGetErrorString(hipGetLastError()));
            return ok ? ms : -1.f;
        };
        const bool found = tuner().pick(key, measure, pick, n_chains, kTrialSteps);
        if (mst) return mst;
        if (!found) return DSDP_OK;   // no candidate fits: the fixed rule decides
    }
    const DockCandidate dc = dock_candidate(pick);
    use = layout(dc.form);
    if (mst) return mst;
    waves = dc.waves;
    return DSDP_OK;
}

// dsdp_dock on a workspace that is either the caller's (d_ws, ws_bytes) or, with
// d_ws NULL, the library's static scratch of this device.
dsdp_status dock_impl(dsdp_grids g, const dsdp_ligand *lig, int32_t n_chains, int32_t n_steps, uint64_t seed,
                      const dsdp_params *prm, int32_t top_k, void *d_ws, size_t ws_bytes, void *stream,
                      dsdp_pose *out, float *out_xyz, int32_t *n_out, dsdp_pose *chains_out,
                      dsdp_dock_stats *stats, bool static_ws)
{
    if (n_out) *n_out = 0;
    if (!g) return fail(DSDP_ERR_INVALID_ARG, "grids handle is NULL");
    if (n_chains < 1) return fail(DSDP_ERR_INVALID_ARG, "n_chains %d < 1", n_chains);
    if (n_chains > 65536) return fail(DSDP_ERR_UNSUPPORTED, "n_chains %d > 65536", n_chains);
    if (n_steps < 0) return fail(DSDP_ERR_INVALID_ARG, "n_steps < 0");
    if (top_k < 0 || top_k > n_chains) return fail(DSDP_ERR_INVALID_ARG, "top_k %d outside 0..n_chains", top_k);
    if (top_k > 0 && (!out || !n_out)) return fail(DSDP_ERR_INVALID_ARG, "out/n_out is NULL");
    dsdp_status st = check_params(prm);
    if (!st) st = check_work(prm, n_steps);
    if (st) return st;
    Prepared pl0, alt;
    st = prepare_ligand(lig, g->map_of_type, pl0, intra_ctx(prm, n_chains, false));
    if (st) return st;
    const SearchParams sp = to_search(prm);
    hipStream_t s = (hipStream_t)stream;
    if (static_ws) HIP_TRY(static_scratch(&d_ws), "static scratch address");
    // layout and waves: the tuner's (the static entry point only reads its
    // cache: it measures nothing), else the fixed rule
    const Prepared *use = &pl0;
    int waves = 0;
    dsdp_params dp;
    if (!prm) {
        dsdp_params_default(&dp);
        prm = &dp;
    }
    if (prm->tune == 1 && prm->waves_per_chain == 0 && prm->intra_form == DSDP_INTRA_AUTO && n_steps > 0 && d_ws &&
        aligned256(d_ws)) {
        st = tune_dock(g, lig, prm, pl0, alt, n_chains, seed, sp, (char *)d_ws,
                       static_ws ? kStaticScratchBytes : ws_bytes, s, static_ws, use, waves);
        if (st) return st;
    }
    const Prepared &pl = *use;
    if (waves == 0) {
        st = pick_waves(prm, pl.h, n_chains, waves);
        if (st) return st;
    }
    const SearchWs w = search_ws(pl.h, n_chains);
    if (static_ws) {
        if (w.total > kStaticScratchBytes)
            return fail(DSDP_ERR_UNSUPPORTED, "this dock needs %zu bytes of scratch; the static scratch holds %zu",
                        w.total, kStaticScratchBytes);
        ws_bytes = kStaticScratchBytes;
    }
    if (!d_ws || ws_bytes < w.total) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
    if (!aligned256(d_ws)) return fail(DSDP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    char *ws = (char *)d_ws;
    st = upload_dock(g, pl, w, n_chains, n_steps, seed, top_k, ws, s);
    if (st) return st;

    Events ev;
    if (stats) {
        HIP_TRY(ev.create(), "event");
        HIP_TRY(hipEventRecord(ev.e[0], s), "event");
    }
    float *rec = (float *)(ws + w.records);
    float4 *bxyz = (float4 *)(ws + w.xyz);
    int *sel = (int *)(ws + w.sel);
    HIP_TRY(launch_tick(search_class(pl.h), waves, search_lds_bytes(pl.h, waves),
                        (const uint32_t *)(ws + w.arena), (const ChainTask *)(ws + w.tasks), n_chains,
                        (const GridView *)(ws + w.grids), sp, n_steps, 1, (float *)(ws + w.state), rec, bxyz, s),
            "search launch");
    if (stats) HIP_TRY(hipEventRecord(ev.e[1], s), "event");
    HIP_TRY(launch_rank(rec, bxyz, (const RankSeg *)(ws + w.segs), 1, n_chains, sp.rmsd_cluster, sel, s), "rank launch");
    if (stats) HIP_TRY(hipEventRecord(ev.e[2], s), "event");
    std::vector<float> h_rec((size_t)n_chains * kRecWords);
    std::vector<int> h_sel((size_t)top_k + 1);
    HIP_TRY(hipMemcpyAsync(h_rec.data(), rec, h_rec.size() * 4, hipMemcpyDeviceToHost, s), "result copy");
    HIP_TRY(hipMemcpyAsync(h_sel.data(), sel, h_sel.size() * 4, hipMemcpyDeviceToHost, s), "result copy");
    std::vector<float4> h_xyz;
    if (out_xyz && top_k > 0) {
        h_xyz.resize((size_t)n_chains * kXyzStride);
        HIP_TRY(hipMemcpyAsync(h_xyz.data(), bxyz, h_xyz.size() * 16, hipMemcpyDeviceToHost, s), "result copy");
    }
    HIP_TRY(hipStreamSynchronize(s), "dock");
    const int nt = pl.h.n_tors;
    const int cnt = top_k > 0 ? h_sel[0] : 0;
    for (int q = 0; q < cnt; q++) {
        const int c = h_sel[1 + q];
        fill_pose(&h_rec[(size_t)c * kRecWords], nt, c, out[q]);
        if (out_xyz)
            for (int a = 0; a < pl.h.n_atoms; a++) {
                const float4 v = h_xyz[(size_t)c * kXyzStride + a];
                float *o = out_xyz + ((size_t)q * pl.h.n_atoms + a) * 3;
                o[0] = v.x; o[1] = v.y; o[2] = v.z;
            }
    }
    if (n_out) *n_out = cnt;
    if (chains_out)
        for (int c = 0; c < n_chains; c++) fill_pose(&h_rec[(size_t)c * kRecWords], nt, c, chains_out[c]);
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        add_stats(h_rec.data(), n_chains, stats);
        float ms = 0, ms_search = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[2]), "event");
        HIP_TRY(hipEventElapsedTime(&ms_search, ev.e[0], ev.e[1]), "event");
        stats->kernel_ms = ms;
        stats->search_ms = ms_search;
    }
    return DSDP_OK;
}
}  // namespace

extern "C" {

dsdp_status dsdp_dock(dsdp_grids g, const dsdp_ligand *lig, int32_t n_chains, int32_t n_steps, uint64_t seed,
                      const dsdp_params *prm, int32_t top_k, void *d_ws, size_t ws_bytes, void *stream,
                      dsdp_pose *out, float *out_xyz, int32_t *n_out, dsdp_pose *chains_out,
                      dsdp_dock_stats *stats)
{
    return dock_impl(g, lig, n_chains, n_steps, seed, prm, top_k, d_ws, ws_bytes, stream, out, out_xyz, n_out,
                     chains_out, stats, false);
}

dsdp_status dsdp_dock_static(dsdp_grids g, const dsdp_ligand *lig, int32_t n_chains, int32_t n_steps, uint64_t seed,
                             const dsdp_params *prm, int32_t top_k, void *stream, dsdp_pose *out, float *out_xyz,
                             int32_t *n_out, dsdp_pose *chains_out, dsdp_dock_stats *stats)
{
    return dock_impl(g, lig, n_chains, n_steps, seed, prm, top_k, nullptr, 0, stream, out, out_xyz, n_out,
                     chains_out, stats, true);
}

}  // extern "C"

namespace {

// One launch of a batch plan: a kernel variant and wave count, the LDS its
// largest member needs, its chains (contiguous in the task table).
struct BatchGroup {
    int cls = 0, waves = 1;
    size_t lds = 0;
    long first = 0, count = 0;
};
struct BatchPlan {
    std::vector<BatchGroup> groups;
    std::vector<int> order;                // ligands in task-table order
    std::vector<const Prepared *> blob;    // each ligand's blob in the plan's layout
};

// The plan of candidate `c`: each ligand's layout from its pair class, one
// launch per (kernel variant, waves); waves lowered for a launch whose largest
// member does not fit the LDS.  Returns false when a ligand cannot run.
bool tuned_plan(int c, const std::vector<Prepared> &pp, const std::vector<Prepared> &pa, int n_chains, BatchPlan &out)
{
    const Plan pl = plan(c);
    out = BatchPlan();
    const int n = (int)pp.size();
    out.blob.resize((size_t)n);
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int l = 0; l < n; l++) {
        const Prepared &pr = plan_form(pl, pp[(size_t)l].h.n_pairs) == DSDP_INTRA_PAIRS ? pp[(size_t)l] : pa[(size_t)l];
        out.blob[(size_t)l] = &pr;
        groups[{search_class(pr.h), pl.waves}].push_back(l);
    }
    for (auto &kv : groups) {
        BatchGroup b;
        b.cls = kv.first.first;
        b.waves = kv.first.second;
        for (;;) {
            b.lds = 0;
            for (int l : kv.second) b.lds = std::max(b.lds, search_lds_bytes(out.blob[(size_t)l]->h, b.waves));
            if (b.lds <= device_max_lds() || b.waves == 1) break;
            b.waves--;
        }
        if (b.lds > device_max_lds()) return false;
        // the largest ligands' chains first, so that the launch ends on short work
        std::vector<int> mem = kv.second;
        std::stable_sort(mem.begin(), mem.end(), [&](int a, int c) {
            const LigHeader &ha = out.blob[(size_t)a]->h, &hc = out.blob[(size_t)c]->h;
            return ha.n_atoms + ha.n_pairs > hc.n_atoms + hc.n_pairs;
        });
        b.first = (long)out.order.size() * n_chains;
        b.count = (long)mem.size() * n_chains;
        for (int l : mem) out.order.push_back(l);
        out.groups.push_back(b);
    }
    return true;
}

// Upload a plan's host-written sections: blobs, tasks in the plan's order, the
// grid view, ranking segments.
dsdp_status upload_plan(const BatchPlan &bp, const dsdp_grids_s *g, const uint64_t *seeds, int n_chains, int n_steps,
                        int top_k, const SearchWs &w, char *ws, hipStream_t s)
{
    const int n_ligs = (int)bp.blob.size();
    HostImage img(w.host_end);
    std::vector<uint32_t> blob_off((size_t)n_ligs);
    size_t o = 0;
    for (int l = 0; l < n_ligs; l++) {
        blob_off[(size_t)l] = (uint32_t)o;
        std::memcpy(img.at<uint32_t>(w.arena) + o, bp.blob[(size_t)l]->blob.data(), bp.blob[(size_t)l]->blob.size() * 4);
        o += bp.blob[(size_t)l]->blob.size();
    }
    ChainTask *tasks = img.at<ChainTask>(w.tasks);
    long ti = 0;
    for (int l : bp.order)
        for (int c = 0; c < n_chains; c++, ti++) {
            ChainTask &t = tasks[ti];
            t.blob_off = blob_off[(size_t)l];
            t.blob_words = (uint32_t)bp.blob[(size_t)l]->h.total_words;
            t.chain = (uint32_t)c;
            t.n_steps = n_steps;
            t.seed_lo = (uint32_t)seeds[l];
            t.seed_hi = (uint32_t)(seeds[l] >> 32);
            t.grid = 0;
            t.slot = (int)((long)l * n_chains + c);
            t.fresh = 0;
        }
    GridView view;
    dsdp_status st = device_view(g, ws, w, img.bytes.data(), s, view);
    if (st) return st;
    *img.at<GridView>(w.grids) = view;
    RankSeg *segs = img.at<RankSeg>(w.segs);
    for (int l = 0; l < n_ligs; l++) {
        segs[l].slot0 = l * n_chains;
        segs[l].n_chains = n_chains;
        segs[l].n_atoms = bp.blob[(size_t)l]->h.n_atoms;
        segs[l].top_k = top_k;
        segs[l].sel_off = l * (n_chains + 1);
    }
    HIP_TRY(hipMemcpyAsync(ws, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice, s), "task upload");
    HIP_TRY(hipStreamSynchronize(s), "task upload");
    return DSDP_OK;
}

// Streams and events of a plan's branches (one stream per launch group), released
// on every return path.
struct Branches {
    std::vector<hipStream_t> s;
    std::vector<hipEvent_t> e;   // one per group, then the fork event
    ~Branches()
    {
        for (auto x : s)
            if (x) (void)hipStreamDestroy(x);
        for (auto x : e)
            if (x) (void)hipEventDestroy(x);
    }
    hipError_t make(int n)
    {
        s.assign((size_t)n, nullptr);
        e.assign((size_t)n + 1, nullptr);
        for (auto &x : s)
            if (hipError_t r = hipStreamCreateWithFlags(&x, hipStreamNonBlocking)) return r;
        for (auto &x : e)
            if (hipError_t r = hipEventCreateWithFlags(&x, hipEventDisableTiming)) return r;
        return hipSuccess;
    }
};

// Ticks of a plan from stream `cs`: each group's ticks on its own branch (the
// groups are independent, so one group's tail overlaps the others' work), joined
// back on `cs`.  Used for trials and inside the batch's graph capture.
hipError_t launch_plan(const BatchPlan &bp, Branches &br, const SearchWs &w, char *ws, const SearchParams &sp,
                       int spt, int n_ticks, hipStream_t cs, bool fresh = true)
{
    const int nb = (int)bp.groups.size();
    hipError_t le = hipEventRecord(br.e[(size_t)nb], cs);
    for (int i = 0; i < nb && le == hipSuccess; i++) {
        const BatchGroup &b = bp.groups[(size_t)i];
        le = hipStreamWaitEvent(br.s[(size_t)i], br.e[(size_t)nb], 0);
        for (int k = 0; k < n_ticks && le == hipSuccess; k++)
            le = launch_tick(b.cls, b.waves, b.lds, (const uint32_t *)(ws + w.arena),
                             (const ChainTask *)(ws + w.tasks) + b.first, (int)b.count,
                             (const GridView *)(ws + w.grids), sp, spt, (k == 0 && fresh) ? 1 : 0, (float *)(ws + w.state),
                             (float *)(ws + w.records), (float4 *)(ws + w.xyz), br.s[(size_t)i]);
        if (le == hipSuccess) le = hipEventRecord(br.e[(size_t)i], br.s[(size_t)i]);
        if (le == hipSuccess) le = hipStreamWaitEvent(cs, br.e[(size_t)i], 0);
    }
    return le;
}

}  // namespace

extern "C" {

int32_t dsdp_tune_entries(dsdp_tune_entry *out, int32_t cap)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const std::vector<TuneEntry> v = tuner().entries(dev);
    for (int i = 0; out && i < cap && i < (int)v.size(); i++) {
        dsdp_tune_entry &o = out[i];
        const TuneEntry &e = v[(size_t)i];
        std::memset(&o, 0, sizeof o);
        o.device = e.key.device;
        o.kind = e.key.kind;
        o.chains = e.key.chains;
        o.shapes = (int32_t)e.key.shapes.size();
        o.plan = e.pick;
        if (e.key.kind == kTuneBatch) {
            const Plan p = plan(e.pick);
            o.intra_form_small = p.form_small;
            o.intra_form_large = p.form_large;
            o.waves_per_chain = p.waves;
        } else {
            const DockCandidate d = dock_candidate(e.pick);
            o.intra_form_small = o.intra_form_large = d.form;
            o.waves_per_chain = d.waves;
        }
        o.trial_steps = e.trial_steps;
        for (int c = 0; c < DSDP_TUNE_CANDIDATES && c < (int)e.trial_ms.size(); c++)
            o.trial_ms[c] = e.trial_ms[(size_t)c];
    }
    return (int32_t)v.size();
}

void dsdp_tune_reset(void) { tuner().clear(); }

size_t dsdp_dock_batch_workspace_bytes(const dsdp_ligand *ligs, int32_t n_ligs, int32_t n_chains)
{
    if (!ligs || n_ligs < 1 || n_chains < 1) return 0;
    size_t words = 0;
    for (int l = 0; l < n_ligs; l++) {
        const size_t lw = max_blob_words(&ligs[l]);
        if (lw == 0) return 0;
        words += lw;
    }
    // blobs sized for either layout, so the tuner's plan does not change the size
    return search_ws(words, (long)n_ligs * n_chains, 1, n_ligs).total;
}

dsdp_status dsdp_dock_batch(dsdp_grids g, const dsdp_ligand *ligs, int32_t n_ligs, int32_t n_chains, int32_t n_steps,
                            const uint64_t *seeds, const dsdp_params *prm, int32_t top_k, int32_t steps_per_tick,
                            void *d_ws, size_t ws_bytes, void *stream, dsdp_pose *out, int32_t *n_out,
                            dsdp_dock_stats *stats)
{
    if (!g) return fail(DSDP_ERR_INVALID_ARG, "grids handle is NULL");
    if (!ligs || n_ligs < 1 || !seeds) return fail(DSDP_ERR_INVALID_ARG, "ligands/seeds missing");
    if (n_chains < 1 || n_chains > 65536) return fail(DSDP_ERR_INVALID_ARG, "n_chains %d outside 1..65536", n_chains);
    if ((long)n_ligs * n_chains > (1L << 24)) return fail(DSDP_ERR_UNSUPPORTED, "more than 2^24 chains in one batch");
    if (n_steps < 0 || steps_per_tick < 0) return fail(DSDP_ERR_INVALID_ARG, "negative step count");
    if (top_k < 0 || top_k > n_chains) return fail(DSDP_ERR_INVALID_ARG, "top_k %d outside 0..n_chains", top_k);
    if (top_k > 0 && (!out || !n_out)) return fail(DSDP_ERR_INVALID_ARG, "out/n_out is NULL");
    dsdp_status st = check_params(prm);
    if (!st) st = check_work(prm, n_steps);
    if (st) return st;
    dsdp_params def;
    dsdp_params_default(&def);
    const dsdp_params &pp = prm ? *prm : def;
    const bool tune = pp.tune == 1 && pp.optimizer == DSDP_OPT_BFGS && pp.waves_per_chain == 0 &&
                      pp.intra_form == DSDP_INTRA_AUTO && n_steps > 0;
    // every ligand prepared in the fixed rule's layout (atom lists for a mixed
    // launch, unless the caller fixed one) and, when tuning, in the other one
    std::vector<Prepared> pls((size_t)n_ligs), alt(tune ? (size_t)n_ligs : 0);
    size_t words = 0;
    for (int l = 0; l < n_ligs; l++) {
        st = prepare_ligand(&ligs[l], g->map_of_type, pls[(size_t)l], intra_ctx(prm, (long)n_ligs * n_chains, true));
        if (!st && tune) {
            const int other = pls[(size_t)l].h.intra_form == kFormPairs ? DSDP_INTRA_ATOMS : DSDP_INTRA_PAIRS;
            st = prepare_ligand(&ligs[l], g->map_of_type, alt[(size_t)l], IntraCtx{other});
        }
        if (st) {
            char msg[600];
            snprintf(msg, sizeof msg, "ligand %d: %s", l, g_error.c_str());
            return fail(st, "%s", msg);
        }
        words += max_blob_words(&ligs[l]);
    }
    const long n_slots = (long)n_ligs * n_chains;
    const SearchWs w = search_ws(words, n_slots, 1, n_ligs);
    if (!d_ws || ws_bytes < w.total) return fail(DSDP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes", w.total);
    if (!aligned256(d_ws)) return fail(DSDP_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const SearchParams sp = to_search(prm);
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream");
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{cs};

    BatchPlan bp;
    if (tune) {
        // the fixed rule's layout is in pls, the other in alt
        const bool pls_atoms = pls[0].h.intra_form == kFormAtoms;
        const std::vector<Prepared> &pp_pairs = pls_atoms ? alt : pls, &pp_atoms = pls_atoms ? pls : alt;
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev), "device");
        std::vector<ShapeBucket> shapes((size_t)n_ligs);
        for (int l = 0; l < n_ligs; l++)
            shapes[(size_t)l] = shape_bucket(pls[(size_t)l].h.n_atoms, pls[(size_t)l].h.n_pairs, 6 + pls[(size_t)l].h.n_tors);
        const TuneKey key = tune_key(dev, n_chains, shapes);
        dsdp_status mst = DSDP_OK;
        // a trial: the candidate's plan over every chain of the batch, one
        // untimed step from fresh starts (so that no candidate pays a kernel's
        // first-launch costs in its time, nor times the chains' first steps)
        // and then the next kTrialSteps steps timed (the search afterwards
        // starts afresh)
        auto measure = [&](int c) -> float {
            BatchPlan tp;
            if (mst || !tuned_plan(c, pp_pairs, pp_atoms, n_chains, tp)) return -1.f;
            // 1 + kTrialSteps steps whatever the batch's length, so that batches of
            // any length share the cached pick
            if ((mst = upload_plan(tp, g, seeds, n_chains, 1 + kTrialSteps, top_k, w, ws, cs))) return -1.f;
            Branches br;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            float ms = -1.f;
            bool ok = br.make((int)tp.groups.size()) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
                      hipEventCreate(&e1) == hipSuccess && launch_plan(tp, br, w, ws, sp, 1, 1, cs) == hipSuccess &&
                      hipEventRecord(e0, cs) == hipSuccess &&
                      launch_plan(tp, br, w, ws, sp, kTrialSteps, 1, cs, false) == hipSuccess &&
                      hipEventRecord(e1, cs) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                      hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (!ok) mst = fail(DSDP_ERR_DEVICE, "tuner trial: %s", hipGetErrorString(hipGetLastError()));
            return ok ? ms : -1.f;
        };
        int pick = 0;
        const bool found = tuner().pick(key, measure, pick, n_slots, kTrialSteps);
        if (mst) return mst;
        if (!found || !tuned_plan(pick, pp_pairs, pp_atoms, n_chains, bp))
            return fail(DSDP_ERR_UNSUPPORTED, "no launch plan fits the batch");
    } else {
        std::vector<const LigHeader *> hdr((size_t)n_ligs);
        std::vector<long> ch((size_t)n_ligs, n_chains);
        for (int l = 0; l < n_ligs; l++) hdr[(size_t)l] = &pls[(size_t)l].h;
        std::vector<LaunchGroup> groups;
        st = plan_groups(prm, hdr, ch, groups);
        if (st) return st;
        bp.blob.resize((size_t)n_ligs);
        for (int l = 0; l < n_ligs; l++) bp.blob[(size_t)l] = &pls[(size_t)l];
        for (const LaunchGroup &lg : groups) {
            BatchGroup b;
            b.cls = lg.cls;
            b.waves = lg.waves;
            b.lds = lg.lds;
            b.first = (long)bp.order.size() * n_chains;
            b.count = lg.chains;
            for (int l : lg.members) bp.order.push_back(l);
            bp.groups.push_back(b);
        }
    }
    st = upload_plan(bp, g, seeds, n_chains, n_steps, top_k, w, ws, s);
    if (st) return st;

    // ticks of steps_per_tick MC steps (0: about eight ticks), captured once as a
    // graph: each group's ticks on its own branch, then the ranking
    const int spt = steps_per_tick > 0 ? steps_per_tick : std::max(1, (n_steps + 7) / 8);
    const int n_ticks = n_steps > 0 ? (n_steps + spt - 1) / spt : 1;
    float *rec = (float *)(ws + w.records);
    float4 *bxyz = (float4 *)(ws + w.xyz);
    int *sel = (int *)(ws + w.sel);
    Branches br;
    HIP_TRY(br.make((int)bp.groups.size()), "stream");
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "graph capture");
    hipError_t le = launch_plan(bp, br, w, ws, sp, spt, n_ticks, cs);
    if (le == hipSuccess) le = launch_rank(rec, bxyz, (const RankSeg *)(ws + w.segs), n_ligs, n_chains, sp.rmsd_cluster, sel, cs);
    hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "batch launch");
    }
    HIP_TRY(ce, "graph capture");
    hipGraphExec_t exec = nullptr;
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(ie, "graph instantiate");
    struct ExecGuard {
        hipGraphExec_t e;
        ~ExecGuard() { (void)hipGraphExecDestroy(e); }
    } eguard{exec};
    Events ev;
    if (stats) {
        HIP_TRY(ev.create(), "event");
        HIP_TRY(hipEventRecord(ev.e[0], s), "event");
    }
    HIP_TRY(hipGraphLaunch(exec, s), "graph launch");
    if (stats) {
        HIP_TRY(hipEventRecord(ev.e[1], s), "event");
        HIP_TRY(hipEventRecord(ev.e[2], s), "event");
    }
    std::vector<float> h_rec((size_t)n_slots * kRecWords);
    std::vector<int> h_sel((size_t)n_slots + n_ligs);
    HIP_TRY(hipMemcpyAsync(h_rec.data(), rec, h_rec.size() * 4, hipMemcpyDeviceToHost, s), "result copy");
    HIP_TRY(hipMemcpyAsync(h_sel.data(), sel, h_sel.size() * 4, hipMemcpyDeviceToHost, s), "result copy");
    HIP_TRY(hipStreamSynchronize(s), "batch");
    for (int l = 0; l < n_ligs; l++) {
        const int *sl = &h_sel[(size_t)l * (n_chains + 1)];
        const int cnt = top_k > 0 ? sl[0] : 0;
        for (int q = 0; q < cnt; q++) {
            const int c = sl[1 + q];
            fill_pose(&h_rec[((size_t)l * n_chains + c) * kRecWords], pls[(size_t)l].h.n_tors, c,
                      out[(size_t)l * top_k + q]);
        }
        if (n_out) n_out[l] = cnt;
    }
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        add_stats(h_rec.data(), n_slots, stats);
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[2]), "event");
        stats->kernel_ms = ms;
        stats->search_ms = ms;
    }
    return DSDP_OK;
}

}  // extern "C"
