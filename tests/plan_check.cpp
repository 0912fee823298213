// plan_check.cpp -- host-only checks of the planner (jt_plan.cpp), built by
// tests/test_plan_sanitized.py with AddressSanitizer and UndefinedBehavior-
// Sanitizer.  Reads a tree and per-slot evidence from a text file, compiles
// the plan, builds the per-propagation schedule for several active-slot
// counts and checks that
//   * every work-list entry and slot set stays inside its list and region;
//   * every collect task runs for the evidence-free slot (when shared) and for
//     exactly the (task, slot) pairs with evidence of that slot below it;
//   * every distribute (task, active slot) pair runs exactly once, either in
//     a multi-slot set (only when the slot reads a shared source) or alone;
//   * the collect sources point at the slot itself or at the shared slot;
//   * the per-launch byte counts add up to the propagation's.
// Prints "OK <summary>" or "FAIL <reason>" and exits non-zero on failure.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "jt_plan.h"

namespace {

int fail(const std::string &m) {
    std::printf("FAIL %s\n", m.c_str());
    return 1;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 2) return fail("usage: plan_check FILE");
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return fail("cannot open input");
    auto rd = [&](long long &x) { return std::fscanf(f, "%lld", &x) == 1; };
    long long nv, nc, ns, nvars_total, tb, gmin;
    if (!rd(nv)) return fail("input");
    std::vector<int32_t> card(nv);
    for (auto &c : card) { long long x; rd(x); c = (int32_t)x; }
    rd(nc);
    std::vector<int64_t> off(nc + 1);
    for (auto &o : off) { long long x; rd(x); o = x; }
    rd(nvars_total);
    std::vector<int32_t> cv(nvars_total);
    for (auto &v : cv) { long long x; rd(x); v = (int32_t)x; }
    std::vector<int32_t> parent(nc);
    for (auto &p : parent) { long long x; rd(x); p = (int32_t)x; }
    rd(ns);
    rd(tb);
    rd(gmin);
    std::vector<std::vector<int32_t>> ev((size_t)ns + 1);
    for (long long s = 0; s < ns; ++s) {
        long long k;
        rd(k);
        for (long long a = 0; a < k; ++a) { long long x; rd(x); ev[s].push_back((int32_t)x); }
    }
    std::fclose(f);
    jt_tuning tun{(int32_t)gmin, 0, 0, (int32_t)tb, 0};
    jt_tree_desc d{(int32_t)nv, card.data(), (int32_t)nc, off.data(), cv.data(), parent.data(), (int32_t)ns, &tun};
    jt::Plan P;
    std::string err;
    const jt_status rc = jt::compile_plan(&d, P, err);
    if (rc != JT_OK) return fail("compile_plan: " + err);
    // schedule orientation and dirty sets, recomputed here independently
    std::vector<std::vector<int32_t>> holders(nv);
    for (int32_t c = 0; c < nc; ++c)
        for (int64_t k = off[c]; k < off[c + 1]; ++k) holders[cv[k]].push_back(c);
    // the dataflow check rejects a schedule whose launches are out of order:
    // the collect sweep's last launch moved to the front reads messages no
    // earlier launch finalized (single-slot plans: a batched plan's work
    // lists are laid out in launch order, which the reordering would break
    // first)
    {
        std::string why;
        if (!jt::check_plan(P, why)) return fail("compiled plan rejected: " + why);
        int32_t last_collect = -1;
        for (size_t k = 0; k < P.fused.size(); ++k)
            if (P.fused[k].collect && P.fused[k].count > 0) last_collect = (int32_t)k;
        if (last_collect > 0 && !P.share) {
            jt::Plan Q = P;
            std::rotate(Q.fused.begin(), Q.fused.begin() + last_collect, Q.fused.begin() + last_collect + 1);
            if (jt::check_plan(Q, why)) return fail("reordered schedule accepted");
            if (why.find("before it is finalized") == std::string::npos && why.find("out of order") == std::string::npos)
                return fail("reordered schedule rejected for another reason: " + why);
        }
    }
    long long n_multi_sets = 0, n_multi_pairs = 0, n_single = 0;
    for (int32_t na : {1, 2, (int32_t)std::max<long long>(1, ns / 2), (int32_t)ns}) {
        if (na < 1 || na > ns) continue;
        jt::Dynamic D;
        jt::build_dynamic(P, ev, na, D);
        const int32_t N = P.n_slots;
        int64_t lsum = 0;
        for (int64_t b : D.launch_bytes) lsum += b;
        if (D.launch_bytes.size() != P.fused.size() || lsum != D.bytes) return fail("launch bytes");
        std::vector<std::vector<char>> dirty(na, std::vector<char>(nc, 0));
        for (int32_t s = 0; s < na; ++s) {
            dirty[s][P.root] = 1;
            for (int32_t v : ev[s]) {
                int32_t h = holders[v].empty() ? -1 : holders[v][0];
                for (int32_t c = h; c >= 0 && !dirty[s][c]; c = P.iparent[c]) dirty[s][c] = 1;
            }
        }
        for (int32_t s = 0; s < P.n_regions; ++s)
            for (int32_t c = 0; c < nc; ++c) {
                const int32_t x = D.csrc[(size_t)s * P.csrc_stride + c];
                if (x != s && !(D.shared && s < na && x == N && !dirty[s][c])) return fail("collect source");
                if (D.shared && s < na && !dirty[s][c] && x != N) return fail("clean clique not shared");
            }
        for (const jt::Launch &l : P.fused) {
            if (!l.listed || l.count == 0) continue;
            const int32_t cnt = D.count[l.work_idx], grid = D.grid[l.work_idx];
            if (cnt < 0 || cnt > l.work_cap || grid < cnt || grid > std::max(1, l.work_cap) || grid < 1)
                return fail("count or grid");
            if (l.work_off + l.work_cap > P.work_total) return fail("work region");
            std::map<std::pair<int32_t, int32_t>, int> seen;
            for (int32_t e = 0; e < cnt; ++e) {
                const JtWork w = D.work[l.work_off + e];
                if (l.multi) {
                    if (w.task == -1) continue;
                    if (w.task < 0 || w.task >= l.count) return fail("multi task");
                    if (w.slot < l.chunk_off || w.slot >= l.chunk_off + l.chunk_cap) return fail("chunk index");
                    const JtChunk &ch = D.chunks[w.slot];
                    if (ch.s[0] < 0) return fail("empty set");
                    const int32_t c = P.items[P.tasks[l.begin + w.task].item].clique;
                    bool tail = false;
                    for (int k = 0; k < JT_MS; ++k) {
                        if (ch.s[k] < 0) { tail = true; continue; }
                        if (tail) return fail("set not packed");
                        if (ch.s[k] >= na) return fail("set slot");
                        if (D.csrc[(size_t)ch.s[k] * P.csrc_stride + c] == ch.s[k]) return fail("set slot not shared");
                        if (seen[{w.task, ch.s[k]}]++) return fail("pair twice (multi)");
                        ++n_multi_pairs;
                    }
                    ++n_multi_sets;
                } else {
                    if (w.task == -1) continue;   // per-XCD padding
                    if (w.task < 0 || w.task >= l.count) return fail("task");
                    if (!(w.slot >= 0 && (w.slot < na || (l.collect && w.slot == N && D.shared)))) return fail("slot");
                    if (seen[{w.task, w.slot}]++) return fail("pair twice");
                    ++n_single;
                }
            }
            if (l.collect) {
                for (int32_t t = 0; t < l.count; ++t) {
                    const int32_t c = P.items[P.tasks[l.begin + t].item].clique;
                    for (int32_t s = 0; s < na; ++s) {
                        const bool want = D.shared ? dirty[s][c] : true;
                        if ((seen.count({t, s}) > 0) != want) return fail("collect pair coverage");
                    }
                    if (D.shared && !seen.count({t, N})) return fail("evidence-free task missing");
                }
            }
        }
        // distribute: multi + single launches of one level cover every pair once
        for (size_t k = 0; k < P.fused.size(); ++k) {
            const jt::Launch &l = P.fused[k];
            if (!l.listed || l.collect || l.multi || l.count == 0) continue;
            std::map<std::pair<int32_t, int32_t>, int> cover;
            std::vector<const jt::Launch *> pair{&l};
            if (k > 0 && P.fused[k - 1].multi && P.fused[k - 1].begin == l.begin) pair.push_back(&P.fused[k - 1]);
            for (const jt::Launch *m : pair)
                for (int32_t e = 0; e < D.count[m->work_idx]; ++e) {
                    const JtWork w = D.work[m->work_off + e];
                    if (w.task < 0) continue;
                    if (m->multi) {
                        for (int kk = 0; kk < JT_MS; ++kk)
                            if (D.chunks[w.slot].s[kk] >= 0) cover[{w.task, D.chunks[w.slot].s[kk]}]++;
                    } else if (w.task >= 0) {
                        cover[{w.task, w.slot}]++;
                    }
                }
            for (int32_t t = 0; t < l.count; ++t)
                for (int32_t s = 0; s < na; ++s)
                    if (cover[{t, s}] != 1) return fail("distribute pair coverage");
            if ((int64_t)cover.size() != (int64_t)l.count * na) return fail("distribute extra pairs");
        }
        // a one-slot distribute launch not marked after_multi runs before the
        // side stream's multi-slot launches are joined: none of its pairs may
        // have its parent pass in a multi-slot set
        std::set<std::pair<int32_t, int32_t>> multi_pair;   // (clique, slot)
        for (const jt::Launch &l : P.fused) {
            if (!l.listed || !l.multi) continue;
            for (int32_t e = 0; e < D.count[l.work_idx]; ++e) {
                const JtWork w = D.work[l.work_off + e];
                if (w.task < 0) continue;
                const int32_t c = P.items[P.tasks[l.begin + w.task].item].clique;
                for (int kk = 0; kk < JT_MS; ++kk)
                    if (D.chunks[w.slot].s[kk] >= 0) multi_pair.insert({c, D.chunks[w.slot].s[kk]});
            }
        }
        for (const jt::Launch &l : P.fused) {
            if (!l.listed || l.collect || l.multi || l.after_multi) continue;
            for (int32_t e = 0; e < D.count[l.work_idx]; ++e) {
                const JtWork w = D.work[l.work_off + e];
                if (w.task < 0) continue;
                const int32_t c = P.items[P.tasks[l.begin + w.task].item].clique;
                const int32_t p = P.iparent[c];
                if (p >= 0 && multi_pair.count({p, w.slot})) return fail("one-slot pass after a multi-slot parent pass, unjoined");
                if (D.shared && p >= 0 && !dirty[w.slot][c]) return fail("one-slot pass without evidence below, unjoined");
            }
        }
    }
    std::printf("OK multi_sets=%lld multi_pairs=%lld single=%lld\n", n_multi_sets, n_multi_pairs, n_single);
    return 0;
}
