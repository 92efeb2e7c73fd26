// jk_prof.hip -- kernel timing hook (include/jk_prof.h).
#include <hip/hip_runtime.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/jk_prof.h"
#include "jk_kernels.hpp"

namespace {

struct Rec {
    const char *name;
    int pair;
};

struct Prof {
    bool on = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev;   // 2 per pair
    std::vector<Rec> recs;
    int64_t dropped = 0;
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<int64_t> cnt;
};

Prof &prof()
{
    static Prof p;
    return p;
}

} // namespace

namespace jk {

void ProfScope::set_capturing(bool on) { prof().capturing = on; }

ProfScope::ProfScope(const char *name, hipStream_t s) : stream_(s), pair_(-1)
{
    Prof &p = prof();
    if (!p.on || p.capturing)
        return;
    const int npair = (int)(p.ev.size() / 2);
    const int next = (int)p.recs.size();
    if (next >= npair) {
        p.dropped++;
        return;
    }
    if (hipEventRecord(p.ev[2 * next], s) != hipSuccess)
        return;
    pair_ = next;
    p.recs.push_back(Rec{name, next});
}

ProfScope::~ProfScope()
{
    if (pair_ < 0)
        return;
    (void)hipEventRecord(prof().ev[2 * pair_ + 1], stream_);
}

} // namespace jk

extern "C" {

int jk_prof_enable(int32_t capacity)
{
    Prof &p = prof();
    if (capacity <= 0) {
        p.on = false;
        return 0;
    }
    if ((int)p.ev.size() < 2 * capacity) {
        for (hipEvent_t e : p.ev)
            (void)hipEventDestroy(e);
        p.ev.assign(2 * (size_t)capacity, nullptr);
        for (auto &e : p.ev)
            if (hipEventCreate(&e) != hipSuccess)
                return -1;
    }
    p.recs.clear();
    p.dropped = 0;
    p.on = true;
    return 0;
}

void jk_prof_reset(void)
{
    prof().recs.clear();
    prof().dropped = 0;
}

int32_t jk_prof_collect(void)
{
    Prof &p = prof();
    p.names.clear();
    p.ms.clear();
    p.cnt.clear();
    for (const Rec &r : p.recs) {
        if (hipEventSynchronize(p.ev[2 * r.pair + 1]) != hipSuccess)
            return -1;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.ev[2 * r.pair], p.ev[2 * r.pair + 1]) != hipSuccess)
            return -1;
        size_t i = 0;
        while (i < p.names.size() && p.names[i] != r.name)
            i++;
        if (i == p.names.size()) {
            p.names.emplace_back(r.name);
            p.ms.push_back(0.0);
            p.cnt.push_back(0);
        }
        p.ms[i] += t;
        p.cnt[i] += 1;
    }
    return (int32_t)p.names.size();
}

int jk_prof_entry(int32_t i, const char **name, double *total_ms, int64_t *launches)
{
    Prof &p = prof();
    if (i < 0 || (size_t)i >= p.names.size())
        return -1;
    if (name)
        *name = p.names[i].c_str();
    if (total_ms)
        *total_ms = p.ms[i];
    if (launches)
        *launches = p.cnt[i];
    return 0;
}

int64_t jk_prof_dropped(void) { return prof().dropped; }

} // extern "C"
