// Launch-variant autotuner.  A tuned site offers a few launch variants of one
// kernel (tile edge, threads per matrix, work order) that compute the same
// bits, so the choice changes speed only.  The first call with a new shape
// key times every variant once on the call's own data (each leaves the same
// outputs) and keeps the fastest: per process, and in the text file named by
// ZS_AUTOTUNE_CACHE when that is set (read once, appended on every new
// choice).  ZS_AUTOTUNE=0, zs_autotune(0), graph capture and the
// no-allocation query path use cached choices or the site's default and time
// nothing.
#include "zoomsvd.h"
#include "zs_internal.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

namespace zs {
namespace {

struct Choice {
    int v = 0;
    std::string ms;       // timings of the candidates, for the report
};

std::mutex g_mu;
std::map<std::string, Choice> g_table;   // "site|key" -> choice
std::map<std::string, int> g_forced;     // site -> variant for every key
bool g_loaded = false;
int g_on = -1;                           // -1: from the environment
thread_local bool t_suspended = false;

std::string full_key(const char *site, const char *key) { return std::string(site) + "|" + key; }

const char *cache_path()
{
    const char *p = std::getenv("ZS_AUTOTUNE_CACHE");
    return p && *p ? p : nullptr;
}

// Reads the cache file once (lines "site|key<TAB>choice<TAB>timings").
void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char *t1 = std::strchr(line, '\t');
        if (!t1) continue;
        *t1 = 0;
        const int v = std::atoi(t1 + 1);
        char *t2 = std::strchr(t1 + 1, '\t');
        Choice c;
        c.v = v;
        if (t2) {
            c.ms = t2 + 1;
            while (!c.ms.empty() && (c.ms.back() == '\n' || c.ms.back() == '\r')) c.ms.pop_back();
        }
        g_table[line] = c;
    }
    std::fclose(f);
}

}  // namespace

int tune_bucket(int64_t n)
{
    int b = 1;
    while (b < n && b < (1 << 30)) b *= 2;
    return b;
}

bool tune_enabled()
{
    if (t_suspended) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_on < 0) {
        const char *e = std::getenv("ZS_AUTOTUNE");
        g_on = (e && e[0] == '0') ? 0 : 1;
    }
    return g_on == 1;
}

void tune_suspend(bool on) { t_suspended = on; }
bool tune_suspended() { return t_suspended; }

int tune_lookup(const char *site, const char *key)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto f = g_forced.find(site);
    if (f != g_forced.end()) return f->second;
    load_locked();
    auto it = g_table.find(full_key(site, key));
    return it == g_table.end() ? -1 : it->second.v;
}

void tune_record(const char *site, const char *key, int choice, const float *ms, int n)
{
    std::string times;
    for (int i = 0; i < n; ++i) {
        char b[32];
        std::snprintf(b, sizeof b, "%s%.4f", i ? "," : "", ms[i]);
        times += b;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    const std::string k = full_key(site, key);
    Choice c;
    c.v = choice;
    c.ms = times;
    g_table[k] = c;
    if (const char *path = cache_path()) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s\t%d\t%s\n", k.c_str(), choice, times.c_str());
            std::fclose(f);
        }
    }
}

bool stream_capturing(hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) {
        (void)hipGetLastError();
        return true;                     // unknown: do not time anything
    }
    return st != hipStreamCaptureStatusNone;
}

}  // namespace zs

extern "C" {

void zs_autotune(int on)
{
    std::lock_guard<std::mutex> lk(zs::g_mu);
    zs::g_on = on ? 1 : 0;
}

zs_status zs_autotune_force(const char *site, int variant)
{
    if (!site) return ZS_EINVAL;
    std::lock_guard<std::mutex> lk(zs::g_mu);
    if (variant < 0) zs::g_forced.erase(site);
    else zs::g_forced[site] = variant;
    return ZS_OK;
}

const char *zs_autotune_table(void)
{
    static thread_local std::string out;
    std::lock_guard<std::mutex> lk(zs::g_mu);
    zs::load_locked();
    out.clear();
    for (auto &kv : zs::g_table) {
        out += kv.first;
        out += "\t";
        out += std::to_string(kv.second.v);
        out += "\t";
        out += kv.second.ms;
        out += "\n";
    }
    return out.c_str();
}

}  // extern "C"
