// The batched kernel's configuration per device (which compiled variant:
// messages per mask-table group and waves per SIMD, and the grid
// multiplier), and the autotuner's cache file: JSON, one entry per device
// kind, keyed by the GPU's architecture name and compute-unit count.
//
// File layout (written by cache_save, one entry per line so that a line
// scanner reads it back; other entries are kept when one is rewritten):
//   {"format": "tdes-batch-tune-1", "entries": [
//   {"device": "gfx950:sramecc+:xnack-", "cus": 256, "kmax": 8, "waves": 4, "grid_mult": 2, "us_per_batch": 207.1},
//   ...
//   ]}
#include <errno.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace tdes {

namespace {

constexpr int kMaxDevices = 64;
constexpr const char *kFormat = "tdes-batch-tune-1";

// Packed per-device configuration: 0 = not chosen yet; else
// kmax | waves << 8 | grid_mult << 16.
std::atomic<uint32_t> g_cfg[kMaxDevices];
std::mutex g_cfg_mu;

uint32_t pack(const BatchConfig &c) {
    return (uint32_t)c.kmax | (uint32_t)c.waves << 8 | (uint32_t)c.grid_mult << 16;
}
BatchConfig unpack(uint32_t v) {
    return BatchConfig{(int)(v & 0xff), (int)(v >> 8 & 0xff), (int)(v >> 16 & 0xff)};
}

struct Entry {
    std::string device;
    long cus = 0;
    BatchConfig cfg{};
    double us = 0;
};

// The value after "key": in line (a string in quotes, or a number).
bool field_str(const std::string &line, const char *key, std::string *out) {
    const std::string k = std::string("\"") + key + "\":";
    size_t p = line.find(k);
    if (p == std::string::npos) return false;
    p = line.find('"', p + k.size());
    if (p == std::string::npos) return false;
    const size_t q = line.find('"', p + 1);
    if (q == std::string::npos) return false;
    *out = line.substr(p + 1, q - p - 1);
    return true;
}

bool field_num(const std::string &line, const char *key, double *out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t p = line.find(k);
    if (p == std::string::npos) return false;
    const char *s = line.c_str() + p + k.size();
    char *end = nullptr;
    errno = 0;
    const double v = strtod(s, &end);
    if (end == s || errno != 0) return false;
    *out = v;
    return true;
}

bool parse_entry(const std::string &line, Entry *e) {
    double cus, kmax, waves, mult, us = 0;
    if (!field_str(line, "device", &e->device) || !field_num(line, "cus", &cus) ||
        !field_num(line, "kmax", &kmax) || !field_num(line, "waves", &waves) ||
        !field_num(line, "grid_mult", &mult))
        return false;
    (void)field_num(line, "us_per_batch", &us);
    e->cus = (long)cus;
    e->cfg = BatchConfig{(int)kmax, (int)waves, (int)mult};
    e->us = us;
    return true;
}

// Entries of the file at path (none if it is missing or unreadable; lines
// that are not entries are ignored).
std::vector<Entry> read_entries(const std::string &path) {
    std::vector<Entry> v;
    FILE *f = fopen(path.c_str(), "r");
    if (f == nullptr) return v;
    std::string line;
    char buf[512];
    while (fgets(buf, sizeof buf, f) != nullptr) {
        line += buf;
        if (line.empty() || line.back() != '\n') continue;  // a long line: keep reading
        Entry e;
        if (line.find("\"device\":") != std::string::npos && parse_entry(line, &e)) v.push_back(e);
        line.clear();
    }
    Entry e;
    if (line.find("\"device\":") != std::string::npos && parse_entry(line, &e)) v.push_back(e);
    fclose(f);
    return v;
}

bool make_parent_dirs(const std::string &path) {
    for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1)) {
        const std::string d = path.substr(0, p);
        if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return false;
    }
    return true;
}

bool name_ok(const char *s) {
    if (s == nullptr || *s == '\0' || strlen(s) > 200) return false;
    for (; *s; s++)
        if (*s == '"' || *s == '\\' || (unsigned char)*s < 0x20) return false;
    return true;
}

// Architecture name and compute units of device dev.
bool device_identity(int dev, std::string *arch, int *cus) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return false;
    *arch = p.gcnArchName;
    *cus = p.multiProcessorCount;
    return name_ok(arch->c_str()) && *cus > 0;
}

}  // namespace

std::string tune_cache_path() {
    const char *env = getenv("TDES_TUNE_CACHE");
    if (env != nullptr) return env;  // "" switches the cache off
    const char *xdg = getenv("XDG_CACHE_HOME");
    if (xdg != nullptr && *xdg) return std::string(xdg) + "/tdes/batch_tune.json";
    const char *home = getenv("HOME");
    if (home != nullptr && *home) return std::string(home) + "/.cache/tdes/batch_tune.json";
    return "";
}

int cache_load(const char *path, const char *device, long cus, BatchConfig *out) {
    if (path == nullptr || *path == '\0' || !name_ok(device) || out == nullptr) return -1;
    for (const Entry &e : read_entries(path)) {
        if (e.device == device && e.cus == cus && batch_config_valid(e.cfg)) {
            *out = e.cfg;
            return 1;
        }
    }
    return 0;
}

bool cache_save(const char *path, const char *device, long cus, const BatchConfig &c,
                double us_per_batch) {
    if (path == nullptr || *path == '\0' || !name_ok(device) || !batch_config_valid(c)) return false;
    std::vector<Entry> v = read_entries(path);
    bool replaced = false;
    for (Entry &e : v) {
        if (e.device == device && e.cus == cus) {
            e.cfg = c;
            e.us = us_per_batch;
            replaced = true;
        }
    }
    if (!replaced) v.push_back(Entry{device, cus, c, us_per_batch});
    if (!make_parent_dirs(path)) return false;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (f == nullptr) return false;
    bool ok = fprintf(f, "{\"format\": \"%s\", \"entries\": [\n", kFormat) > 0;
    for (size_t i = 0; i < v.size() && ok; i++)
        ok = fprintf(f,
                     "{\"device\": \"%s\", \"cus\": %ld, \"kmax\": %d, \"waves\": %d, "
                     "\"grid_mult\": %d, \"us_per_batch\": %.3f}%s\n",
                     v[i].device.c_str(), v[i].cus, v[i].cfg.kmax, v[i].cfg.waves,
                     v[i].cfg.grid_mult, v[i].us, i + 1 < v.size() ? "," : "") > 0;
    ok = ok && fprintf(f, "]}\n") > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        unlink(tmp.c_str());
        return false;
    }
    return true;
}

hipError_t batch_config_current(BatchConfig *out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    uint32_t v = g_cfg[dev].load(std::memory_order_acquire);
    if (v == 0) {
        // first use on this device: the cached tuning result, else the default
        std::lock_guard<std::mutex> lock(g_cfg_mu);
        v = g_cfg[dev].load(std::memory_order_relaxed);
        if (v == 0) {
            BatchConfig c = batch_config_default();
            std::string arch;
            int cus = 0;
            const std::string path = tune_cache_path();
            BatchConfig cached;
            if (!path.empty() && device_identity(dev, &arch, &cus) &&
                cache_load(path.c_str(), arch.c_str(), cus, &cached) == 1)
                c = cached;
            v = pack(c);
            g_cfg[dev].store(v, std::memory_order_release);
        }
    }
    *out = unpack(v);
    return hipSuccess;
}

hipError_t batch_config_set(const BatchConfig &c) {
    if (!batch_config_valid(c)) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    g_cfg[dev].store(pack(c), std::memory_order_release);
    return hipSuccess;
}

bool batch_config_persist(const BatchConfig &c, double us_per_batch) {
    const std::string path = tune_cache_path();
    if (path.empty()) return true;  // cache switched off
    int dev = 0;
    std::string arch;
    int cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || !device_identity(dev, &arch, &cus)) return false;
    return cache_save(path.c_str(), arch.c_str(), cus, c, us_per_batch);
}

}  // namespace tdes
