// Launch-plan tuner of the search: plain C++, no device code, so its selection
// and cache logic can be unit-tested on the host.  Private to the library.
//
// A batch's launch plan says, for every ligand, which layout of the
// intra-ligand term its blob uses and how many waves each of its chains gets;
// ligands with the same kernel variant and wave count share a launch.  A single
// ligand's dock has the same two choices, layout and waves.  The candidates
// (kPlans for batches, kDockCandidates for docks) are fixed; for a request not
// yet in the cache of the current device, the caller's `measure` callback
// times every candidate on a short trial of that request (all of its chains, a
// few steps) and the fastest is cached by the request's make-up: the kind of
// request, the histogram of ligand shapes (heavy atoms, intra-ligand pairs,
// tangent dimension) and the chain count.  Candidates the callback reports as
// impossible (negative time) are skipped.  Search results do not depend on the
// choice, so the tuner only moves speed.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace dsdp {
namespace host {

// A ligand's shape bucket: heavy atoms rounded up to a multiple of 8, pair-list
// size class (512, 1024 or 2048 pairs at most), more than 16 tangent coordinates.
struct ShapeBucket {
    int atoms = 0, pairs = 0, wide = 0;
    bool operator<(const ShapeBucket &o) const
    {
        return std::tie(atoms, pairs, wide) < std::tie(o.atoms, o.pairs, o.wide);
    }
};

inline ShapeBucket shape_bucket(int n_atoms, int n_pairs, int dim)
{
    ShapeBucket b;
    b.atoms = ((std::max(n_atoms, 1) + 7) / 8) * 8;
    b.pairs = n_pairs <= 512 ? 512 : (n_pairs <= 1024 ? 1024 : 2048);
    b.wide = dim > 16 ? 1 : 0;
    return b;
}

inline int round_up_pow2(long v)
{
    int p = 1;
    while (p < v && p < (1 << 30)) p <<= 1;
    return p;
}

// Kinds of tuned request (their candidates differ).
enum TuneKind { kTuneBatch = 0, kTuneDockBfgs = 1, kTuneDockBb = 2 };

// The cache key of a request: device, kind, ligand-shape histogram (each
// bucket's count rounded up to a power of two, so that batches of about the
// same make-up share an entry), chains per ligand.
struct TuneKey {
    int device = 0;
    int kind = kTuneBatch;
    int chains = 0;
    std::vector<std::pair<ShapeBucket, int>> shapes;   // sorted by bucket
    bool operator<(const TuneKey &o) const
    {
        if (device != o.device) return device < o.device;
        if (kind != o.kind) return kind < o.kind;
        if (chains != o.chains) return chains < o.chains;
        if (shapes.size() != o.shapes.size()) return shapes.size() < o.shapes.size();
        for (size_t i = 0; i < shapes.size(); i++) {
            if (shapes[i].first < o.shapes[i].first) return true;
            if (o.shapes[i].first < shapes[i].first) return false;
            if (shapes[i].second != o.shapes[i].second) return shapes[i].second < o.shapes[i].second;
        }
        return false;
    }
    bool operator==(const TuneKey &o) const { return !(*this < o) && !(o < *this); }
};

inline TuneKey tune_key(int device, int chains, const std::vector<ShapeBucket> &ligands, int kind = kTuneBatch)
{
    std::map<ShapeBucket, int> h;
    for (const ShapeBucket &b : ligands) h[b]++;
    TuneKey k;
    k.device = device;
    k.kind = kind;
    k.chains = chains;
    for (const auto &kv : h) k.shapes.push_back({kv.first, round_up_pow2(kv.second)});
    return k;
}

// The candidate plans: for each, the layout of a ligand's intra-ligand term as
// a function of its pair class (1 pair lists, 2 atom lists) and the waves per
// chain.  Plan 0 is the library's fixed rule for batches that fill the device.
struct Plan {
    int form_small;   // layout of ligands with at most 512 pairs
    int form_large;   // layout of ligands with more
    int waves;
};
constexpr int kPlans = 6;
inline Plan plan(int i)
{
    static const Plan p[kPlans] = {
        {2, 2, 1},   // atom lists, one wave per chain
        {2, 2, 2},   // atom lists, two waves
        {1, 1, 1},   // pair lists, one wave
        {1, 1, 2},   // pair lists, two waves
        {1, 2, 1},   // pair lists for small pair sets, atom lists for the rest, one wave
        {1, 2, 2},   // the same, two waves
    };
    return p[(i >= 0 && i < kPlans) ? i : 0];
}
inline int plan_form(const Plan &p, int n_pairs) { return n_pairs <= 512 ? p.form_small : p.form_large; }

// The candidates of a single ligand's dock: both layouts (1 pair lists, 2 atom
// lists) at 4, 3, 2 and 1 waves per chain.
struct DockCandidate {
    int form;
    int waves;
};
constexpr int kDockCandidates = 8;
inline DockCandidate dock_candidate(int i)
{
    const int c = (i >= 0 && i < kDockCandidates) ? i : 0;
    return {c < 4 ? 1 : 2, 4 - (c & 3)};
}
inline int candidates_of(int kind) { return kind == kTuneBatch ? kPlans : kDockCandidates; }

struct TuneEntry {
    TuneKey key;
    int pick = 0;                 // index into the kind's candidates
    std::vector<float> trial_ms;  // per candidate (< 0: could not run)
    int trial_steps = 0;
    long trial_chains = 0;
};

class Tuner {
public:
    // measure(plan index) -> trial milliseconds, or < 0 when the plan cannot run.
    using Measure = std::function<float(int)>;

    // The cached pick of `key`, else the fastest of its kind's candidates by
    // `measure` (ties to the lower index), cached.  Returns false when no
    // candidate can run.
    bool pick(const TuneKey &key, const Measure &measure, int &out, long trial_chains = 0, int trial_steps = 0)
    {
        if (find(key, out)) return true;
        TuneEntry e;
        e.key = key;
        e.trial_chains = trial_chains;
        e.trial_steps = trial_steps;
        float best = -1.f;
        const int n = candidates_of(key.kind);
        for (int c = 0; c < n; c++) {
            const float t = measure(c);
            e.trial_ms.push_back(t >= 0.f ? t : -1.f);
            if (!(t >= 0.f)) continue;
            if (best < 0.f || t < best) {
                best = t;
                e.pick = c;
            }
        }
        if (best < 0.f) return false;
        std::lock_guard<std::mutex> lock(mu_);
        auto it = cache_.find(key);   // another thread may have tuned it meanwhile: keep the first
        if (it == cache_.end()) it = cache_.emplace(key, e).first;
        out = it->second.pick;
        return true;
    }

    // The cached pick of `key`, if any (counted as a hit); measures nothing.
    bool find(const TuneKey &key, int &out)
    {
        std::lock_guard<std::mutex> lock(mu_);
        auto it = cache_.find(key);
        if (it == cache_.end()) return false;
        out = it->second.pick;
        hits_++;
        return true;
    }

    std::vector<TuneEntry> entries(int device) const
    {
        std::lock_guard<std::mutex> lock(mu_);
        std::vector<TuneEntry> v;
        for (const auto &kv : cache_)
            if (kv.first.device == device) v.push_back(kv.second);
        return v;
    }

    void clear()
    {
        std::lock_guard<std::mutex> lock(mu_);
        cache_.clear();
        hits_ = 0;
    }

    long hits() const
    {
        std::lock_guard<std::mutex> lock(mu_);
        return hits_;
    }

private:
    mutable std::mutex mu_;
    std::map<TuneKey, TuneEntry> cache_;
    long hits_ = 0;
};

}  // namespace host
}  // namespace dsdp
