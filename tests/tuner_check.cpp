// Host unit check of the search's launch tuner (bucket keys, request kinds,
// candidate plans of batches and docks, selection and cache logic) with a
// scripted measurement in place of trial launches.  Built and run by tests/test_tuner.py with
// AddressSanitizer and UBSan.
#include "tuner.h"

#include <cstdio>
#include <thread>
#include <vector>

using namespace dsdp::host;

static int failures = 0;
#define CHECK(c)                                                                      \
    do {                                                                              \
        if (!(c)) {                                                                   \
            std::fprintf(stderr, "tuner check failed: %s (line %d)\n", #c, __LINE__); \
            failures++;                                                               \
        }                                                                             \
    } while (0)

int main()
{
    // shape buckets: atoms to multiples of 8, pair classes, more than 16 tangent coordinates
    {
        const ShapeBucket a = shape_bucket(20, 150, 10);
        CHECK(a.atoms == 24 && a.pairs == 512 && a.wide == 0);
        const ShapeBucket b = shape_bucket(25, 513, 17);
        CHECK(b.atoms == 32 && b.pairs == 1024 && b.wide == 1);
        CHECK(shape_bucket(60, 1800, 37).pairs == 2048 && shape_bucket(1, 0, 6).atoms == 8);
        CHECK(round_up_pow2(1) == 1 && round_up_pow2(3) == 4 && round_up_pow2(4096) == 4096 && round_up_pow2(4097) == 8192);
    }
    // batch keys: the histogram of shapes with counts rounded up to powers of
    // two, in bucket order, whatever the ligand order; chains and device count
    {
        const ShapeBucket s1 = shape_bucket(20, 150, 10), s2 = shape_bucket(50, 900, 20);
        const TuneKey k1 = tune_key(0, 128, {s1, s2, s1});
        const TuneKey k2 = tune_key(0, 128, {s2, s1, s1});
        CHECK(k1 == k2 && k1.shapes.size() == 2 && k1.shapes[0].second == 2 && k1.shapes[1].second == 1);
        const TuneKey k3 = tune_key(0, 128, {s1, s1, s1, s2});   // 3 -> 4 ligands of s1: another make-up
        CHECK(!(k3 == k1) && k3.shapes[0].second == 4);
        const TuneKey k4 = tune_key(0, 128, {s1, s1, s1, s1, s2});   // 4 rounds alike
        CHECK(k4 == k3);
        CHECK(!(tune_key(0, 64, {s1, s2, s1}) == k1) && !(tune_key(1, 128, {s1, s2, s1}) == k1));
        // the kind of request is part of the key
        const TuneKey d1 = tune_key(0, 128, {s1}, kTuneDockBfgs), d2 = tune_key(0, 128, {s1}, kTuneDockBb);
        CHECK(!(d1 == d2) && !(d1 == tune_key(0, 128, {s1})) && d1 == tune_key(0, 128, {s1}, kTuneDockBfgs));
    }
    // dock candidates: pair lists at 4, 3, 2, 1 waves, then atom lists alike
    {
        CHECK(kDockCandidates == 8 && candidates_of(kTuneBatch) == kPlans && candidates_of(kTuneDockBb) == 8);
        const int form[8] = {1, 1, 1, 1, 2, 2, 2, 2}, waves[8] = {4, 3, 2, 1, 4, 3, 2, 1};
        for (int i = 0; i < 8; i++) CHECK(dock_candidate(i).form == form[i] && dock_candidate(i).waves == waves[i]);
        CHECK(dock_candidate(-1).waves == 4 && dock_candidate(8).form == 1);
    }
    // candidate plans: plan 0 is the fixed rule (atom lists, one wave); the
    // layout of a ligand follows its pair class
    {
        CHECK(kPlans == 6);
        const Plan p0 = plan(0), p4 = plan(4);
        CHECK(p0.form_small == 2 && p0.form_large == 2 && p0.waves == 1);
        CHECK(plan_form(p4, 512) == 1 && plan_form(p4, 513) == 2 && p4.waves == 1);
        CHECK(plan(5).waves == 2 && plan(-1).waves == p0.waves && plan(99).form_small == p0.form_small);
    }
    // selection: the fastest runnable plan, ties to the lower index; cached
    {
        Tuner t;
        int calls = 0;
        const TuneKey k = tune_key(0, 128, {shape_bucket(32, 355, 13)});
        auto m = [&](int c) -> float {
            calls++;
            if (c == 3) return -1.f;   // cannot run
            if (c == 2 || c == 4) return 3.0f;
            return 5.0f + c;
        };
        int p = -1;
        CHECK(t.pick(k, m, p, 65536, 3));
        CHECK(p == 2 && calls == kPlans);
        CHECK(t.pick(k, m, p) && p == 2 && calls == kPlans && t.hits() == 1);   // cached: no new trial
        const std::vector<TuneEntry> e = t.entries(0);
        CHECK(e.size() == 1 && e[0].pick == 2 && e[0].trial_ms.size() == (size_t)kPlans && e[0].trial_ms[3] < 0.f &&
              e[0].trial_ms[2] == 3.0f && e[0].trial_chains == 65536 && e[0].trial_steps == 3);
        CHECK(t.entries(1).empty());
        const TuneKey k1 = tune_key(1, 128, {shape_bucket(32, 355, 13)});   // another device measures again
        CHECK(t.pick(k1, m, p) && calls == 2 * kPlans && t.entries(1).size() == 1);
        // a dock key of the same shape is another entry, over the dock candidates
        const TuneKey kd = tune_key(0, 128, {shape_bucket(32, 355, 13)}, kTuneDockBfgs);
        int q = -1;
        CHECK(!t.find(kd, q) && q == -1);
        CHECK(t.pick(kd, [&](int c) { calls++; return c == 6 ? 1.0f : 2.0f; }, q) && q == 6);
        CHECK(calls == 2 * kPlans + kDockCandidates && t.entries(0).size() == 2);
        int r = -1;
        CHECK(t.find(kd, r) && r == 6);   // read from the cache, nothing measured
        CHECK(calls == 2 * kPlans + kDockCandidates);
        t.clear();
        CHECK(t.entries(0).empty() && t.hits() == 0);
    }
    // nothing runnable: no pick, nothing cached
    {
        Tuner t;
        int p = -1;
        CHECK(!t.pick(tune_key(0, 1, {shape_bucket(64, 2000, 37)}), [](int) { return -1.f; }, p));
        CHECK(t.entries(0).empty());
    }
    // concurrent callers of one key: one cached entry, every caller gets it
    {
        Tuner t;
        const TuneKey k = tune_key(0, 512, {shape_bucket(40, 700, 20)});
        std::vector<std::thread> th;
        std::vector<int> got(8, -1);
        for (int i = 0; i < 8; i++)
            th.emplace_back([&, i] { t.pick(k, [](int c) { return (float)(10 - c); }, got[(size_t)i]); });
        for (auto &x : th) x.join();
        CHECK(t.entries(0).size() == 1);
        for (int g : got) CHECK(g == kPlans - 1);
    }
    if (failures) return 1;
    std::printf("tuner: keys, candidate plans, selection, cache and concurrency as specified\n");
    return 0;
}
