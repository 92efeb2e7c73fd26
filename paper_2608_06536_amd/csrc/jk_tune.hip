// jk_tune.hip -- the plan table of include/jk_tune.h: shape-class keys,
// recorded plans, JSON save and load.  Host code only; the timing loop
// (jk_autotune) lives with the build orchestration in jk_api.hip.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cctype>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/jk_tune.h"
#include "jk_tune.hpp"

namespace {

typedef std::tuple<int64_t, int64_t, int32_t, int32_t> Key;   // (nao/64, R/64, precision, packed)

std::mutex g_mu;
std::map<Key, jk_tuning> g_table;

Key key_of(const jk_problem *p)
{
    const int64_t R = p->ndens * p->rank;
    return Key((p->nao + 63) / 64, (R + 63) / 64, p->precision, (p->flags & JK_B_PACKED) ? 1 : 0);
}

bool valid_tuning(const jk_tuning &t)
{
    return t.ht_tile >= 0 && t.ht_tile <= 4 && t.chunk_mb >= 64 && t.chunk_mb <= 4096;
}

// Minimal reader for the flat JSON this file writes: objects of integer
// fields inside an "entries" array.
struct Reader {
    const char *s;
    size_t i = 0;
    void ws()
    {
        while (s[i] && isspace((unsigned char)s[i]))
            i++;
    }
    bool lit(char c)
    {
        ws();
        if (s[i] != c)
            return false;
        i++;
        return true;
    }
    bool str(std::string &out)
    {
        ws();
        if (s[i] != '"')
            return false;
        size_t j = ++i;
        while (s[i] && s[i] != '"')
            i++;
        if (s[i] != '"')
            return false;
        out.assign(s + j, i - j);
        i++;
        return true;
    }
    bool integer(int64_t &v)
    {
        ws();
        size_t j = i;
        if (s[i] == '-')
            i++;
        if (!isdigit((unsigned char)s[i]))
            return false;
        while (isdigit((unsigned char)s[i]))
            i++;
        if (i - j > 18)
            return false;
        v = strtoll(std::string(s + j, i - j).c_str(), nullptr, 10);
        return true;
    }
};

} // namespace

namespace jk {

jk_tuning tuning_for(const jk_problem *p)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(key_of(p));
    if (it != g_table.end())
        return it->second;
    return jk_tuning{4, 1024};
}

void tuning_record(const jk_problem *p, const jk_tuning &t)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key_of(p)] = t;
}

} // namespace jk

extern "C" {

static jk_status jk_tuning_get_impl(const jk_problem *p, jk_tuning *t)
{
    if (!p || !t || jk_workspace_bytes(p) == 0)
        return JK_EINVAL;
    *t = jk::tuning_for(p);
    return JK_OK;
}

jk_status jk_tuning_get(const jk_problem *p, jk_tuning *t)
{
    try {
        return jk_tuning_get_impl(p, t);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static jk_status jk_tuning_set_impl(const jk_problem *p, const jk_tuning *t)
{
    if (!p || !t || !valid_tuning(*t) || jk_workspace_bytes(p) == 0)
        return JK_EINVAL;
    jk::tuning_record(p, *t);
    return JK_OK;
}

jk_status jk_tuning_set(const jk_problem *p, const jk_tuning *t)
{
    try {
        return jk_tuning_set_impl(p, t);
    } catch (...) {
        return JK_ENOMEM;
    }
}

static void jk_tuning_clear_impl(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

void jk_tuning_clear(void)
{
    try {
        jk_tuning_clear_impl();
    } catch (...) {
    }
}

static size_t jk_tuning_save_impl(char *buf, size_t cap)
{
    std::string out = "{\"version\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_mu);
        bool first = true;
        for (const auto &kv : g_table) {
            char line[256];
            snprintf(line, sizeof line,
                     "%s\n  {\"nao64\": %lld, \"rank64\": %lld, \"precision\": %d, \"packed\": %d, "
                     "\"ht_tile\": %d, \"chunk_mb\": %d}",
                     first ? "" : ",", (long long)std::get<0>(kv.first),
                     (long long)std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                     kv.second.ht_tile, kv.second.chunk_mb);
            out += line;
            first = false;
        }
    }
    out += "\n]}\n";
    if (buf && cap > 0) {
        const size_t n = out.size() < cap - 1 ? out.size() : cap - 1;
        memcpy(buf, out.data(), n);
        buf[n] = '\0';
    }
    return out.size() + 1;
}

size_t jk_tuning_save(char *buf, size_t cap)
{
    try {
        return jk_tuning_save_impl(buf, cap);
    } catch (...) {
        return 0;
    }
}

static jk_status jk_tuning_load_impl(const char *json)
{
    if (!json)
        return JK_EINVAL;
    Reader r{json};
    std::string name;
    int64_t v;
    std::vector<std::pair<Key, jk_tuning>> got;
    if (!r.lit('{'))
        return JK_EINVAL;
    bool have_entries = false;
    while (true) {
        if (!r.str(name) || !r.lit(':'))
            return JK_EINVAL;
        if (name == "version") {
            if (!r.integer(v) || v != 1)
                return JK_EINVAL;
        } else if (name == "entries") {
            have_entries = true;
            if (!r.lit('['))
                return JK_EINVAL;
            if (!r.lit(']')) {
                while (true) {
                    if (!r.lit('{'))
                        return JK_EINVAL;
                    int64_t f[6] = {-1, -1, -1, -1, -1, -1};
                    static const char *names[6] = {"nao64", "rank64", "precision", "packed",
                                                   "ht_tile", "chunk_mb"};
                    while (true) {
                        if (!r.str(name) || !r.lit(':') || !r.integer(v))
                            return JK_EINVAL;
                        int idx = -1;
                        for (int q = 0; q < 6; q++)
                            if (name == names[q])
                                idx = q;
                        if (idx < 0 || f[idx] != -1)
                            return JK_EINVAL;
                        f[idx] = v;
                        if (r.lit(','))
                            continue;
                        if (r.lit('}'))
                            break;
                        return JK_EINVAL;
                    }
                    for (int q = 0; q < 6; q++)
                        if (f[q] < 0)
                            return JK_EINVAL;
                    const jk_tuning t{(int32_t)f[4], (int32_t)f[5]};
                    if (!valid_tuning(t) || f[0] < 1 || f[0] > 256 || f[1] < 1 ||
                        f[1] > (1 << 14) || (f[2] != JK_FP64 && f[2] != JK_MIXED) || f[3] > 1)
                        return JK_EINVAL;
                    got.push_back({Key(f[0], f[1], (int32_t)f[2], (int32_t)f[3]), t});
                    if (r.lit(','))
                        continue;
                    if (r.lit(']'))
                        break;
                    return JK_EINVAL;
                }
            }
        } else {
            return JK_EINVAL;
        }
        if (r.lit(','))
            continue;
        if (r.lit('}'))
            break;
        return JK_EINVAL;
    }
    r.ws();
    if (json[r.i] != '\0' || !have_entries)
        return JK_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &e : got)
        g_table[e.first] = e.second;
    return JK_OK;
}

jk_status jk_tuning_load(const char *json)
{
    try {
        return jk_tuning_load_impl(json);
    } catch (...) {
        return JK_ENOMEM;
    }
}

} // extern "C"
