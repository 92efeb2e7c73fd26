// host_abi_check.cpp -- the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitize.py builds the
// library's sources with the sanitizers on their host side, links this driver
// and runs it; no GPU is needed).
//
// Every call here returns before any device work: workspace sizes and plans
// over a grid of shapes (single, batched, packed, mixed), plan descriptions
// under explicit tunings, the tuning table's JSON round trip and its reader
// on malformed text, and the argument checks of every entry point (null
// pointers, misaligned or short workspaces, mismatched batch members).  Exit
// status 0 and a final "ok" line when every status is the one expected.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../include/jk.h"
#include "../include/jk_tune.h"

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        failures++;
    }
}

static jk_problem prob(int64_t nao, int64_t naux, int64_t nd, int64_t r, int prec, int flags)
{
    jk_problem p;
    std::memset(&p, 0, sizeof p);
    p.nao = nao;
    p.naux = naux;
    p.ndens = nd;
    p.rank = r;
    p.precision = prec;
    p.flags = flags;
    return p;
}

int main()
{
    // status strings (the enumerators; the library also reads other values a
    // C caller may pass, which a C++ caller cannot form)
    for (jk_status s : {JK_OK, JK_EINVAL, JK_EWORKSPACE, JK_EUNSUPPORTED, JK_EHIP, JK_ENOMEM})
        expect(jk_status_str(s) != nullptr, "status string");

    // workspace sizes and plans over a grid of shapes
    const int64_t naos[] = {1, 7, 48, 130, 500, 2047};
    const int64_t nauxs[] = {1, 13, 2000};
    const int64_t nds[] = {1, 3, 9, 16};
    const int flagset[] = {0, 1, 2, 3, 4, 5, 6, 7};
    size_t checked = 0;
    for (int64_t nao : naos)
        for (int64_t naux : nauxs)
            for (int64_t nd : nds)
                for (int prec = 0; prec < 2; prec++)
                    for (int fl : flagset) {
                        const int64_t r = nao / 10 + 1;
                        jk_problem p = prob(nao, naux, nd, r, prec, fl);
                        const size_t ws = jk_workspace_bytes(&p);
                        expect(ws > 0, "workspace of a valid problem");
                        jk_plan_info info;
                        expect(jk_plan_describe(&p, nullptr, &info) == JK_OK, "plan of a valid problem");
                        for (int tile : {0, 1, 2, 3, 4})
                            for (int mb : {64, 1024, 4096}) {
                                jk_tuning t{tile, mb};
                                expect(jk_plan_describe(&p, &t, &info) == JK_OK, "plan under a tuning");
                            }
                        if (fl & JK_B_PACKED)
                            continue;
                        expect(jk_fock_workspace_bytes(&p, naux) > 0, "Fock workspace");
                        checked++;
                    }
    // invalid problems
    jk_problem bad[] = {prob(0, 1, 1, 1, 0, 0), prob(5, 0, 1, 1, 0, 0), prob(5, 1, 0, 1, 0, 0),
                        prob(5, 1, 1, 0, 0, 0), prob(5, 1, 1, 6, 0, 0), prob(5, 1, 1, 1, 7, 0),
                        prob(5, 1, 1, 1, 0, 8), prob(5, 1, 1, 1, 0, -1)};
    for (const jk_problem &p : bad)
        expect(jk_workspace_bytes(&p) == 0, "workspace of an invalid problem is 0");
    expect(jk_workspace_bytes(nullptr) == 0, "workspace of a null problem is 0");

    // batched sizes: uneven members, both precisions, packed and not
    for (int prec = 0; prec < 2; prec++)
        for (int fl : {0, 3, 4, 7}) {
            std::vector<jk_problem> ps;
            for (int g = 0; g < 17; g++)
                ps.push_back(prob(1 + 29 * g % 300, 1 + 7 * g, 1 + g % 5, 1 + g % 7, prec, fl));
            for (jk_problem &q : ps)
                if (q.rank > q.nao)
                    q.rank = q.nao;
            expect(jk_batched_workspace_bytes((int32_t)ps.size(), ps.data()) > 0, "batched workspace");
        }
    expect(jk_batched_workspace_bytes(0, nullptr) == 0, "empty batch");

    // the tuning table: set, get, save, clear, load, and malformed text
    {
        jk_problem p = prob(500, 2000, 8, 40, 0, 0);
        jk_tuning t{3, 512}, u{0, 0};
        expect(jk_tuning_set(&p, &t) == JK_OK, "tuning set");
        expect(jk_tuning_get(&p, &u) == JK_OK && u.ht_tile == 3 && u.chunk_mb == 512, "tuning get");
        const size_t need = jk_tuning_save(nullptr, 0);
        std::vector<char> buf(need + 1);
        expect(jk_tuning_save(buf.data(), buf.size()) == need, "tuning save");
        std::vector<char> small(need / 2 + 1);
        jk_tuning_save(small.data(), small.size());          // truncated: must not overrun
        jk_tuning_clear();
        expect(jk_tuning_load(buf.data()) == JK_OK, "tuning load of a saved table");
        expect(jk_tuning_get(&p, &u) == JK_OK && u.ht_tile == 3 && u.chunk_mb == 512,
               "tuning survives the round trip");
        const std::string text(buf.data());
        const char *junk[] = {"", "{", "}", "[", "[{", "{\"entries\":", "{\"entries\":[{]}",
                              "null", "[1,2,3]", "{\"a\":\"\\u12\"}", "{\"entries\":[{\"nao_class\":-1}]}",
                              "\x01\x02\xff"};
        for (const char *j : junk)
            (void)jk_tuning_load(j);                         // any status; no crash, no overrun
        for (size_t cut = 0; cut < text.size(); cut += 7)
            (void)jk_tuning_load(text.substr(0, cut).c_str());
        std::string flipped = text;
        for (size_t i = 0; i < flipped.size(); i += 5) {
            std::string f = flipped;
            f[i] = (char)(f[i] ^ 0x21);
            (void)jk_tuning_load(f.c_str());
        }
        expect(jk_tuning_load(nullptr) != JK_OK, "tuning load of null");
        jk_tuning_clear();
    }

    // argument checks: every entry point refuses before any launch
    {
        jk_problem p = prob(10, 4, 2, 3, 0, 0);
        const size_t need = jk_workspace_bytes(&p);
        const double *d = (const double *)(uintptr_t)256;
        double *o = (double *)(uintptr_t)256;
        void *ws = (void *)(uintptr_t)256;
        expect(jk_build(&p, nullptr, d, d, o, o, ws, need, nullptr) == JK_EINVAL, "build: null B");
        expect(jk_build(&p, d, d, d, o, o, (void *)(uintptr_t)257, need, nullptr) == JK_EINVAL,
               "build: misaligned workspace");
        expect(jk_build(&p, d, d, d, o, o, ws, need - 1, nullptr) == JK_EWORKSPACE,
               "build: short workspace");
        expect(jk_vjp(&p, d, d, d, d, d, o, o, nullptr, ws, need, nullptr) == JK_EINVAL,
               "vjp: one of dCL, dCR");
        expect(jk_vjp(&p, d, d, d, d, d, o, o, o, ws, need - 1, nullptr) == JK_EWORKSPACE,
               "vjp: short workspace");
        const double coef[3] = {2.0, -1.0, 0.0};
        const size_t nf = jk_fock_workspace_bytes(&p, 0);
        expect(jk_fock(&p, d, nullptr, 0, d, d, coef, o, ws, nf - 1, nullptr) == JK_EWORKSPACE,
               "fock: short workspace");
        jk_problem pj = prob(10, 4, 2, 3, 0, JK_WANT_J);
        expect(jk_fock(&pj, d, nullptr, 0, d, d, coef, o, ws, nf, nullptr) == JK_EINVAL,
               "fock: J only");
        jk_problem two[2] = {prob(10, 4, 2, 3, 0, 0), prob(12, 5, 1, 2, 0, JK_WANT_J)};
        const double *pd[2] = {d, d};
        double *po[2] = {o, o};
        expect(jk_build_batched(2, two, pd, pd, pd, po, po, ws, (size_t)1 << 40, nullptr) == JK_EINVAL,
               "batched: members with different flags");
        two[1].flags = 0;
        const size_t nb = jk_batched_workspace_bytes(2, two);
        expect(jk_build_batched(2, two, pd, pd, pd, po, po, ws, nb - 1, nullptr) == JK_EWORKSPACE,
               "batched: short workspace");
        expect(jk_build_batched(0, two, pd, pd, pd, po, po, ws, nb, nullptr) == JK_EINVAL,
               "batched: no members");
        jk_problem mixed5 = prob(10, 4, 2, 3, 1, 0);
        mixed5.nslice = 5;
        const size_t nm = jk_workspace_bytes(&mixed5);
        expect(nm == 0 || jk_build(&mixed5, d, d, d, o, o, ws, nm, nullptr) == JK_EUNSUPPORTED,
               "build: unsupported digit count");
    }

    std::printf("%zu shapes checked\n", checked);
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
