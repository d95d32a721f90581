// Ownership checker of the operation pool (test infrastructure).  After every
// launch that can move chunks (the pass kernels, the detach, the persistent
// kernel) it walks the whole pool on the host and checks that
//   * every chunk id is in exactly one place: the free ring's live range
//     [ring_head, ring_tail), one buffer's main list (head .. tail), one
//     buffer's overflow list, or one work item's chunk list;
//   * no list has a cycle, and a main list ends at the tail its tail word names;
//   * a buffer's count (bcnt) is CH times the chunks it holds;
//   * every counted operation in a (partition, query) buffer targets a vertex
//     of that partition.
// Failures are counted and the first message kept (simt_check_* below).
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "fork_dev.h"

namespace {
fk::GraphDev g_g{};
fk::QueryDev g_q{};
fk::BufDev g_b{};
bool g_have_g = false, g_have_q = false, g_have_b = false;
unsigned long long g_checks = 0, g_fail = 0;
std::string g_msg;
int g_mode = -1;  // SIMT_CHECK: 0 off, 1 on (default)

void failf(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void failf(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ++g_fail;
    if (g_msg.empty()) g_msg = buf;
    fprintf(stderr, "[simt-check] %s\n", buf);
    if (getenv("SIMT_ABORT")) abort();
}

struct Walker {
    std::vector<int64_t> where;  // owner code of each chunk (-1: unseen)
    bool ok = true;
    bool mark(uint32_t id, int64_t code, const char* what) {
        if (id >= where.size()) {
            failf("%s: chunk id %u out of range (pool %zu)", what, id, where.size());
            ok = false;
            return false;
        }
        if (where[id] != -1) {
            failf("%s: chunk %u already owned (code %lld, now %lld)", what, id, (long long)where[id], (long long)code);
            ok = false;
            return false;
        }
        where[id] = code;
        return true;
    }
};

void check_ops(uint32_t ch, uint32_t cnt, uint32_t P, const char* what) {
    const uint32_t v0 = g_g.pstart[P], v1 = g_g.pstart[P + 1];
    if (cnt > (uint32_t)fk::CH) {
        failf("%s: chunk %u counts %u operations", what, ch, cnt);
        return;
    }
    for (uint32_t k = 0; k < cnt; ++k) {
        const uint2 op = g_b.chunks[(unsigned long long)ch * fk::CH + k];
        if (op.x < v0 || op.x >= v1) {
            failf("%s: chunk %u slot %u holds vertex %u outside partition %u [%u, %u)", what, ch, k, op.x, P, v0, v1);
            return;
        }
    }
}

// Planted mistakes (SIMT_PLANT), to show that the checker sees them: after
// the first pass launch whose pool has the needed shape, one chunk is
//   dup     -- listed twice in the free ring (a double free),
//   leak    -- dropped from the free ring (a lost chunk),
//   misroute-- moved from one buffer's main list to a buffer of another
//              partition (operations outside their partition),
//   count   -- counted one chunk short in its buffer's bcnt.
bool plant_once() {
    static bool done = false;
    const char* m = getenv("SIMT_PLANT");
    if (!m || done) return false;
    fk::Ctl* ctl = g_b.ctl;
    const std::string k = m;
    const unsigned long long nch = g_b.nch;
    if ((k == "dup" || k == "leak") && ctl->ring_tail - ctl->ring_head >= 2) {
        if (k == "dup") g_b.ring[(ctl->ring_head + 1) % nch] = g_b.ring[ctl->ring_head % nch];
        else ctl->ring_head += 1;
        done = true;
        return true;
    }
    for (uint32_t P = 0; P < g_g.np && !done; ++P)
        for (uint32_t q = 0; q < g_q.nq && !done; ++q) {
            const unsigned long long b = (unsigned long long)P * g_q.qc + q;
            const int32_t h = g_b.bhead[b];
            const uint32_t tl = (uint32_t)(g_b.btw[b] >> 32);
            if (h < 0) continue;
            if (k == "count") {
                g_b.bcnt[b] -= fk::CH;
                done = true;
            } else if (k == "misroute" && (uint32_t)h != tl && g_b.ccount[h] > 0) {
                // detach the head chunk and give it to the same query's buffer of another partition
                const uint32_t P2 = (P + 1) % g_g.np;
                if (P2 == P) continue;
                const unsigned long long b2 = (unsigned long long)P2 * g_q.qc + q;
                g_b.bhead[b] = g_b.cnext[h];
                g_b.cnext[h] = g_b.bover[b2];
                g_b.bover[b2] = h;
                g_b.bcnt[b2] += fk::CH;
                g_b.bcnt[b] -= fk::CH;
                done = true;
            }
        }
    return done;
}

void check_pool(bool items) {
    const fk::Ctl* ctl = g_b.ctl;
    if (ctl->err) return;  // the run ends with the error; buffers are not kept consistent
    if (!items) plant_once();
    ++g_checks;
    const unsigned long long nch = g_b.nch;
    Walker W;
    W.where.assign(nch, -1);
    if (ctl->ring_tail < ctl->ring_head || ctl->ring_tail - ctl->ring_head > nch) {
        failf("free ring range [%llu, %llu) invalid for %llu chunks", ctl->ring_head, ctl->ring_tail, nch);
        return;
    }
    for (unsigned long long p = ctl->ring_head; p < ctl->ring_tail; ++p)
        if (!W.mark(g_b.ring[p % nch], -2, "ring")) return;
    const uint32_t np = g_g.np, nq = g_q.nq;
    for (uint32_t P = 0; P < np; ++P)
        for (uint32_t q = 0; q < nq; ++q) {
            const unsigned long long b = (unsigned long long)P * g_q.qc + q;
            const int32_t h = g_b.bhead[b], o = g_b.bover[b];
            const unsigned long long w = g_b.btw[b];
            const uint32_t tl = (uint32_t)(w >> 32), f = (uint32_t)w;
            uint64_t n = 0;
            char what[96];
            snprintf(what, sizeof what, "buffer (P %u, q %u) main list", P, q);
            if (h >= 0) {
                int32_t cur = h;
                bool at_tail = false;
                while (cur >= 0) {
                    if (!W.mark((uint32_t)cur, (int64_t)b, what)) return;
                    ++n;
                    const bool is_tail = (uint32_t)cur == tl;
                    check_ops((uint32_t)cur, is_tail ? std::min<uint32_t>(f, fk::CH) : g_b.ccount[cur], P, what);
                    if (is_tail) { at_tail = true; break; }
                    cur = g_b.cnext[cur];
                }
                if (!at_tail) failf("%s: ends at %d before its tail %u", what, cur, tl);
            } else if (tl != 0xffffffffu) {
                failf("%s: empty head but tail word %llx", what, w);
            }
            snprintf(what, sizeof what, "buffer (P %u, q %u) overflow list", P, q);
            for (int32_t cur = o; cur >= 0; cur = g_b.cnext[cur]) {
                if (!W.mark((uint32_t)cur, (int64_t)b, what)) return;
                ++n;
                check_ops((uint32_t)cur, g_b.ccount[cur], P, what);
            }
            if ((uint64_t)g_b.bcnt[b] != n * fk::CH)
                failf("buffer (P %u, q %u): bcnt %u for %llu chunks", P, q, g_b.bcnt[b], (unsigned long long)n);
        }
    if (items) {
        for (uint32_t x = 0; x < (uint32_t)fk::NXCD; ++x) {
            const uint32_t ni = std::min(ctl->nitems[x], g_b.item_cap);
            for (uint32_t k = 0; k < ni; ++k) {
                const fk::Item& it = g_b.items[(unsigned long long)x * g_b.item_cap + k];
                if (it.rest == fk::RESCAN) continue;
                char what[96];
                snprintf(what, sizeof what, "item (P %u, q %u)", it.part, it.q);
                const int64_t code = -1000 - (int64_t)(x * g_b.item_cap + k);
                for (uint32_t j = 0; j < std::min<uint32_t>(it.nch, fk::ICH); ++j) {
                    if (!W.mark(it.ch[j].x, code, what)) return;
                    check_ops(it.ch[j].x, it.ch[j].y, it.part, what);
                }
                for (int32_t cur = it.rest; cur >= 0; cur = g_b.cnext[cur]) {
                    if (!W.mark((uint32_t)cur, code, what)) return;
                    check_ops((uint32_t)cur, g_b.ccount[cur], it.part, what);
                }
            }
        }
    }
    unsigned long long lost = 0, first = 0;
    for (unsigned long long i = 0; i < nch; ++i)
        if (W.where[i] == -1) { if (!lost) first = i; ++lost; }
    if (lost) failf("%llu chunks owned by nothing (first %llu)", lost, first);
}
}  // namespace

namespace simt {
void note_arg(const fk::GraphDev& g) { g_g = g; g_have_g = true; }
void note_arg(const fk::QueryDev& q) { g_q = q; g_have_q = true; }
void note_arg(const fk::BufDev& b) { g_b = b; g_have_b = true; }
void after_launch(const char* name) {
    if (g_mode < 0) g_mode = getenv("SIMT_CHECK") ? atoi(getenv("SIMT_CHECK")) : 1;
    const std::string n = name;
    const bool proc = n.find("k_process") != std::string::npos || n == "cooperative";
    const bool detach = n.find("k_worklist") != std::string::npos;
    // the graph descriptor is kept from the context's last launch that took
    // one (the detach kernel is not given it; its select launch just was)
    if (g_mode && (proc || detach) && g_have_g && g_have_b && g_have_q) check_pool(detach);
    g_have_q = g_have_b = false;
}
}  // namespace simt

extern "C" unsigned long long simt_check_count(void) { return g_checks; }
extern "C" unsigned long long simt_check_failures(void) { return g_fail; }
extern "C" const char* simt_check_message(void) { return g_msg.c_str(); }
extern "C" void simt_check_reset(void) { g_checks = g_fail = 0; g_msg.clear(); }
extern "C" int simt_planted(void) {
    const char* m = getenv("SIMT_PLANT");
    return m && *m ? 1 : 0;
}
