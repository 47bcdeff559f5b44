// Autotuner and learned choice of launch configurations for the stencil
// loop kinds: candidate enumeration, cost-model features, the timing
// database, exhaustive tuning on scratch replicas, training of the cost
// model from the database (the networks of model.cpp, trained on the GPU),
// cost-model files, batched picks and the model -> tuner -> default chain.
//
// The paper names auto-tuning as future work (Sec. "Conclusion"); its
// adaptive rule (Sec. "Adaptive Utilization") is the per-kernel choice from
// profiled times that this generalises to launch shapes and partition
// counts.  Nothing here changes a loop body's arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "jacc.h"

#ifndef JACC_BUILD_ID
#define JACC_BUILD_ID "unversioned"
#endif

namespace {

constexpr int kBlocks[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {64, 4}, {128, 2}, {256, 2}, {256, 4}};
constexpr int kTiles[] = {1, 4, 16, 64};
constexpr int kPersistentTiles[] = {1, 4, 16};
constexpr int kRows3d[] = {1, 4};

bool stencil_kind(int kind, int ndim) {
    return (kind == JACC_LOOP_JACOBI2D && ndim == 2) || (kind == JACC_LOOP_HEAT3D && ndim == 3);
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

std::vector<jacc_candidate> enumerate(int kind, const int64_t *e, int ndim, const int *ks, int nks) {
    std::vector<jacc_candidate> out;
    const bool even = e[ndim - 1] % 2 == 0;
    for (int q = 0; q < nks; ++q) {
        const int K = ks[q];
        if (K > e[0] - 2) continue;  // a partition per interior row at most
        auto add = [&](int bx, int by, int tile, int vec, int pers, int rows) {
            jacc_candidate c{};
            c.cfg.bx = bx;
            c.cfg.by = by;
            c.cfg.tile = tile;
            c.cfg.vec = vec;
            c.cfg.persistent = pers;
            c.cfg.rows = rows;
            c.K = K;
            out.push_back(c);
        };
        for (const auto &b : kBlocks)
            for (int rows : kRows3d) {
                if (rows > 1 && (kind != JACC_LOOP_HEAT3D || b[0] * b[1] > 256)) continue;
                for (int tile : kTiles)
                    for (int vec = 1; vec <= 2; ++vec)
                        if (vec == 1 || even) add(b[0], b[1], tile, vec, 0, rows);
            }
        for (int tile : kPersistentTiles)
            for (int vec = 1; vec <= 2; ++vec)
                if (vec == 1 || even) add(256, 1, tile, vec, 1, 1);
    }
    return out;
}

void features(int kind, const int64_t *e, int ndim, const jacc_candidate &c, float *f) {
    (void)kind;
    const double d0 = (double)e[0], d1 = (double)e[1], d2 = ndim == 3 ? (double)e[2] : 1.0;
    double cells = 1.0;
    for (int d = 0; d < ndim; ++d) cells *= (double)std::max<int64_t>(1, e[d] - 2);
    const int bx = c.cfg.persistent ? 256 : c.cfg.bx, by = c.cfg.persistent ? 1 : c.cfg.by;
    const int rows = c.cfg.rows > 0 ? c.cfg.rows : 1;
    double wg;
    if (ndim == 2)
        wg = (double)cdiv(e[1] - 2, (int64_t)bx * c.cfg.vec) * (double)cdiv(e[0] - 2, (int64_t)by * c.cfg.tile);
    else
        wg = (double)cdiv(e[2] - 2, (int64_t)bx * c.cfg.vec) * (double)cdiv(e[1] - 2, (int64_t)by * rows) *
             (double)cdiv(e[0] - 2, c.cfg.tile);
    const double v[JACC_NFEATURES] = {ndim == 3 ? 1.0 : 0.0,
                                      std::log2(d0),
                                      std::log2(d1),
                                      std::log2(std::max(1.0, d2)),
                                      std::log2(cells),
                                      std::log2((double)c.cfg.bx),
                                      std::log2((double)c.cfg.by),
                                      std::log2((double)c.cfg.tile),
                                      (double)c.cfg.vec,
                                      std::log2((double)c.K),
                                      (double)c.cfg.persistent,
                                      std::log2(std::max(1.0, wg)),
                                      std::log2((double)rows)};
    for (int i = 0; i < JACC_NFEATURES; ++i) f[i] = (float)v[i];
}

double median_of(std::vector<double> s) {
    std::sort(s.begin(), s.end());
    const size_t n = s.size();
    return n % 2 ? s[n / 2] : 0.5 * (s[n / 2 - 1] + s[n / 2]);
}

int argmin_of(const double *v, int n) {
    int best = 0;
    for (int i = 1; i < n; ++i)
        if (v[i] < v[best]) best = i;
    return best;
}

// ---- build key ------------------------------------------------------------
// "<arch>|hip<runtime version>|<build id>" of the current device ("dry" and
// version 0 for a dry-run context); computed once per device.
std::string build_key(jacc_ctx *c) {
    static std::map<int, std::string> keys;  // by device id, -1 for dry-run contexts
    int dev = -1;
    if (!jr::dry(c) && hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        dev = -2;
    }
    auto it = keys.find(dev);
    if (it != keys.end()) return it->second;
    std::string arch = dev == -1 ? "dry" : "unknown";
    int ver = 0;
    if (dev >= 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            const size_t colon = arch.find(':');
            if (colon != std::string::npos) arch.resize(colon);
        }
        (void)hipRuntimeGetVersion(&ver);
        (void)hipGetLastError();
    }
    std::string key = arch + "|hip" + std::to_string(ver) + "|" + JACC_BUILD_ID;
    keys[dev] = key;
    return key;
}

// ---- timing database --------------------------------------------------------
// Text lines: "@ <build key>" opens a section; an entry is
//   <kind> <e0> <e1> <e2> <K> <bx> <by> <tile> <vec> <persistent> <rows> <n> <s_1> ... <s_n>
// (e2 = 0 for 2-D).  '#' starts a comment line.
struct DbKey {
    int kind;
    int64_t e[3];
    int K, bx, by, tile, vec, pers, rows;
    bool operator<(const DbKey &o) const {
        const int64_t a[] = {kind, e[0], e[1], e[2], K, bx, by, tile, vec, pers, rows};
        const int64_t b[] = {o.kind, o.e[0], o.e[1], o.e[2], o.K, o.bx, o.by, o.tile, o.vec, o.pers, o.rows};
        return std::lexicographical_compare(a, a + 11, b, b + 11);
    }
};

struct Db {
    std::map<std::string, std::map<DbKey, std::vector<double>>> sections;  // by build key, in file order of keys
};

DbKey db_key(int kind, const int64_t *e, int ndim, const jacc_candidate &c) {
    DbKey k{};
    k.kind = kind;
    for (int d = 0; d < 3; ++d) k.e[d] = d < ndim ? e[d] : 0;
    k.K = c.K;
    k.bx = c.cfg.bx;
    k.by = c.cfg.by;
    k.tile = c.cfg.tile;
    k.vec = c.cfg.vec;
    k.pers = c.cfg.persistent;
    k.rows = c.cfg.rows;
    return k;
}

// Reads the file into *db (a missing file is an empty database).  Returns an
// error text for a malformed file, else "".
std::string db_read(const char *path, Db *db) {
    std::ifstream f(path);
    if (!f) return "";
    std::string line, section;
    bool have = false;
    int ln = 0;
    while (std::getline(f, line)) {
        ++ln;
        if (line.empty() || line[0] == '#') continue;
        if (line[0] == '@') {
            std::istringstream is(line.substr(1));
            if (!(is >> section)) return "line " + std::to_string(ln) + ": empty section key";
            db->sections[section];
            have = true;
            continue;
        }
        if (!have) return "line " + std::to_string(ln) + ": entry before any section";
        std::istringstream is(line);
        DbKey k{};
        int n = 0;
        if (!(is >> k.kind >> k.e[0] >> k.e[1] >> k.e[2] >> k.K >> k.bx >> k.by >> k.tile >> k.vec >> k.pers >> k.rows >>
              n) ||
            n < 1 || n > 10000)
            return "line " + std::to_string(ln) + ": malformed entry";
        std::vector<double> s((size_t)n);
        for (double &v : s)
            if (!(is >> v) || !(v >= 0.0) || !std::isfinite(v)) return "line " + std::to_string(ln) + ": bad sample";
        std::string extra;
        if (is >> extra) return "line " + std::to_string(ln) + ": trailing text";
        db->sections[section][k] = s;
    }
    return "";
}

bool db_write(const char *path, const Db &db) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "# jacc timing database: kind e0 e1 e2 K bx by tile vec persistent rows n samples(ms)\n";
        char buf[64];
        for (const auto &sec : db.sections) {
            f << "@ " << sec.first << "\n";
            for (const auto &kv : sec.second) {
                const DbKey &k = kv.first;
                f << k.kind << ' ' << k.e[0] << ' ' << k.e[1] << ' ' << k.e[2] << ' ' << k.K << ' ' << k.bx << ' '
                  << k.by << ' ' << k.tile << ' ' << k.vec << ' ' << k.pers << ' ' << k.rows << ' ' << kv.second.size();
                for (double v : kv.second) {
                    snprintf(buf, sizeof buf, " %.17g", v);
                    f << buf;
                }
                f << "\n";
            }
        }
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// ---- scratch replicas ------------------------------------------------------------
// Host copies of the two stencil arrays, entered with another partition count.
struct Replica {
    jacc_ctx *c = nullptr;
    std::vector<double> in, out;
    bool entered_in = false, entered_out = false;
    ~Replica() {
        if (entered_out) (void)jacc_data_exit(c, out.data(), JACC_DELETE);
        if (entered_in) (void)jacc_data_exit(c, in.data(), JACC_DELETE);
    }
};

int make_replica(jacc_ctx *c, const jacc_arg *args, int K, Replica &r) {
    jacc_array_desc d[2];
    size_t bytes[2];
    for (int i = 0; i < 2; ++i) {
        int rc = jr::array_info(c, args[i].host, &d[i], &bytes[i], nullptr);
        if (rc) return rc;
        if (d[i].dtype != JACC_F64) return jr::error(c, JACC_ERR_INVALID, "stencil arrays must be FP64");
    }
    r.c = c;
    r.in.resize(bytes[0] / sizeof(double));
    r.out.resize(bytes[1] / sizeof(double));
    std::memcpy(r.in.data(), args[0].host, bytes[0]);
    std::memcpy(r.out.data(), args[1].host, bytes[1]);
    d[0].num_partitions = K;
    d[1].num_partitions = K;
    int rc = jacc_data_enter(c, r.in.data(), &d[0], JACC_COPYIN);
    if (rc) return rc;
    r.entered_in = true;
    rc = jacc_data_enter(c, r.out.data(), &d[1], JACC_COPYIN);
    if (rc) return rc;
    r.entered_out = true;
    return JACC_OK;
}

// Times one candidate: a graph of `sweeps` captured sweeps, alternating
// between the two scratch arrays, replayed `warmup` times untimed and
// `reps` times timed; ms receives the per-sweep time of each replay (the
// graph launch's own cost spread over the sweeps, so that small loops are
// not timed as launch overhead).
int time_candidate(jacc_ctx *c, int kind, const jacc_bounds *b, const jacc_arg *args, const double *scalars,
                   int nscalars, const jacc_config &cfg, int warmup, int reps, int sweeps, std::vector<double> &ms) {
    int rc = jacc_batch_begin(c);
    if (rc) return rc;
    jacc_arg back[2] = {args[0], args[1]};  // the reverse sweep: out read, in written
    back[0].host = args[1].host;
    back[1].host = args[0].host;
    for (int k = 0; k < sweeps && !rc; ++k)
        rc = jacc_parallel_loop(c, kind, b, 2, (k & 1) ? back : args, scalars, nscalars, -1, nullptr, &cfg);
    int g = -1;
    const int rc_end = jacc_batch_end(c, &g);
    if (!rc) rc = rc_end;
    ms.assign((size_t)reps, 0.0);
    if (!rc) rc = jacc_batch_time(c, g, warmup, reps, ms.data());
    if (!rc)
        for (double &v : ms) v /= sweeps;
    if (g >= 0) {
        const int rc2 = jacc_batch_destroy(c, g);
        if (!rc) rc = rc2;
    }
    return rc;
}

// Sweeps per timed graph: enough that one replay lasts about 0.1 ms (the
// estimate from a one-sweep graph of the first candidate), even, at most 8
// (longer graphs cost more to capture and instantiate than they gain).
int sweeps_for(double one_sweep_ms) {
    if (!(one_sweep_ms > 0)) return 1;
    int n = (int)std::ceil(0.1 / one_sweep_ms);
    if (n <= 1) return 1;
    n = std::min(8, n + (n & 1));
    return n;
}

int loop_shape(jacc_ctx *c, int kind, int nargs, const jacc_arg *args, int64_t *e, int *ndim, int *K) {
    if (!args || nargs != 2) return jr::error(c, JACC_ERR_INVALID, "stencil loops take 2 arguments");
    jacc_array_desc d;
    int rc = jr::array_info(c, args[1].host, &d, nullptr, K);
    if (rc) return rc;
    if (!stencil_kind(kind, d.ndim))
        return jr::error(c, JACC_ERR_UNSUPPORTED, "tuning covers JACOBI2D and HEAT3D loops");
    if (d.part_dim != 0)
        return jr::error(c, JACC_ERR_UNSUPPORTED, "tuning covers arrays split along dimension 0");
    *ndim = d.ndim;
    for (int i = 0; i < d.ndim; ++i) e[i] = d.extent[i];
    return JACC_OK;
}

// ---- cost model: an ensemble of networks plus its scaler ----------------------
struct CostModel {
    jacc_ctx *ctx = nullptr;
    std::string path;
    int F = JACC_NFEATURES;
    std::vector<float> mu, sd;
    std::vector<jacc_model *> nets;
    std::map<std::vector<int64_t>, jacc_config> cache;  // eager picks per loop signature
    ~CostModel() {
        for (jacc_model *m : nets) jacc_model_destroy(m);
    }
};

void release_cost_model(void *p) { delete (CostModel *)p; }

uint64_t fnv1a(const unsigned char *p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t splitmix(uint64_t &s) {  // Steele, Lea, Flood 2014
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// He-uniform weights (limit sqrt(6 / fan_in)), zero biases, output row
// scaled by one half.
std::vector<float> init_params(int F, uint64_t seed) {
    const int H = 64;
    std::vector<float> p;
    uint64_t s = seed;
    auto he = [&](int fan_out, int fan_in, double scale) {
        const double lim = std::sqrt(6.0 / fan_in) * scale;
        for (int i = 0; i < fan_out * fan_in; ++i) {
            const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
            p.push_back((float)(lim * (2.0 * u - 1.0)));
        }
    };
    auto zeros = [&](int n) { p.insert(p.end(), (size_t)n, 0.f); };
    he(H, F, 1.0);
    zeros(H);
    he(H, H, 1.0);
    zeros(H);
    he(H, H, 1.0);
    zeros(H);
    he(1, H, 0.5);
    zeros(1);
    return p;
}

constexpr char kMagic[8] = {'J', 'A', 'C', 'C', 'C', 'M', '0', '1'};

// Reads a model file; returns "" or the reason it was refused.
std::string read_model_file(const char *path, const std::string &key, int *F, int *members, std::vector<float> &mu,
                            std::vector<float> &sd, std::vector<std::vector<float>> &params) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return std::string("cannot open ") + path;
    std::vector<unsigned char> buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (buf.size() < 8 + 4 + 8 || std::memcmp(buf.data(), kMagic, 8) != 0) return "not a cost-model file";
    const size_t body = buf.size() - 8;
    uint64_t sum;
    std::memcpy(&sum, buf.data() + body, 8);
    if (fnv1a(buf.data(), body) != sum) return "checksum mismatch (corrupt or truncated file)";
    size_t o = 8;
    auto take = [&](void *dst, size_t n) {
        if (o + n > body) return false;
        std::memcpy(dst, buf.data() + o, n);
        o += n;
        return true;
    };
    uint32_t klen = 0;
    if (!take(&klen, 4) || klen > 4096) return "bad build-key length";
    std::string fkey(klen, '\0');
    if (!take(&fkey[0], klen)) return "truncated build key";
    if (fkey != key) return "written under build key " + fkey + ", this library is " + key;
    int32_t hdr[2];
    if (!take(hdr, sizeof hdr)) return "truncated header";
    *F = hdr[0];
    *members = hdr[1];
    if (*F != JACC_NFEATURES || *members < 1 || *members > 64) return "bad feature or member count";
    mu.resize((size_t)*F);
    sd.resize((size_t)*F);
    if (!take(mu.data(), mu.size() * 4) || !take(sd.data(), sd.size() * 4)) return "truncated scaler";
    const int P = jacc_model_nparams(*F);
    params.assign((size_t)*members, std::vector<float>((size_t)P));
    for (auto &p : params)
        if (!take(p.data(), p.size() * 4)) return "truncated parameters";
    if (o != body) return "trailing bytes";
    return "";
}

bool write_model_file(const char *path, const std::string &key, int F, const std::vector<float> &mu,
                      const std::vector<float> &sd, const std::vector<std::vector<float>> &params) {
    std::vector<unsigned char> buf(kMagic, kMagic + 8);
    auto put = [&](const void *src, size_t n) {
        const unsigned char *p = (const unsigned char *)src;
        buf.insert(buf.end(), p, p + n);
    };
    const uint32_t klen = (uint32_t)key.size();
    put(&klen, 4);
    put(key.data(), klen);
    const int32_t hdr[2] = {F, (int32_t)params.size()};
    put(hdr, sizeof hdr);
    put(mu.data(), mu.size() * 4);
    put(sd.data(), sd.size() * 4);
    for (const auto &p : params) put(p.data(), p.size() * 4);
    const uint64_t sum = fnv1a(buf.data(), buf.size());
    put(&sum, 8);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return false;
        f.write((const char *)buf.data(), (std::streamsize)buf.size());
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// Builds the networks of a model from host parameters.
int make_nets(jacc_ctx *ctx, CostModel *cm, const std::vector<std::vector<float>> &params) {
    for (const auto &p : params) {
        jacc_model *m = nullptr;
        int rc = jacc_model_create(ctx, cm->F, &m);
        if (rc) return rc;
        cm->nets.push_back(m);
        rc = jacc_model_set_params(m, p.data(), (int)p.size());
        if (!rc) rc = jacc_model_set_scaler(m, cm->mu.data(), cm->sd.data());
        if (rc) return rc;
    }
    return JACC_OK;
}

// Mean prediction of the members over the rows of X (n x F).
int predict(CostModel *cm, const std::vector<float> &X, int n, std::vector<float> &out) {
    out.assign((size_t)n, 0.f);
    std::vector<float> one((size_t)n);
    std::vector<double> acc((size_t)n, 0.0);
    for (jacc_model *m : cm->nets) {
        int rc = jacc_model_predict(m, X.data(), n, one.data());
        if (rc) return rc;
        for (int i = 0; i < n; ++i) acc[i] += one[i];
    }
    for (int i = 0; i < n; ++i) out[i] = (float)(acc[i] / (double)cm->nets.size());
    return JACC_OK;
}

int pick(jacc_ctx *ctx, CostModel *cm, int kind, const int64_t *e, int ndim, const int *ks, int nks,
         bool eager_only, jacc_candidate *best, float *pred, int cap, int *ncand) {
    std::vector<jacc_candidate> cands = enumerate(kind, e, ndim, ks, nks);
    if (eager_only)
        cands.erase(std::remove_if(cands.begin(), cands.end(), [](const jacc_candidate &c) { return c.cfg.persistent; }),
                    cands.end());
    if (cands.empty()) return jr::error(ctx, JACC_ERR_INVALID, "no candidate fits the loop");
    const int n = (int)cands.size();
    std::vector<float> X((size_t)n * cm->F);
    for (int i = 0; i < n; ++i) features(kind, e, ndim, cands[i], &X[(size_t)i * cm->F]);
    std::vector<float> yhat;
    int rc = predict(cm, X, n, yhat);
    if (rc) return rc;
    int b = 0;
    for (int i = 1; i < n; ++i)
        if (yhat[i] < yhat[b]) b = i;
    if (best) *best = cands[b];
    if (pred)
        for (int i = 0; i < n && i < cap; ++i) pred[i] = yhat[i];
    if (ncand) *ncand = n;
    return JACC_OK;
}

int load_model(jacc_ctx *ctx, const char *path) {
    int F = 0, members = 0;
    std::vector<float> mu, sd;
    std::vector<std::vector<float>> params;
    const std::string why = read_model_file(path, build_key(ctx), &F, &members, mu, sd, params);
    if (!why.empty()) {
        jr::attach_model(ctx, nullptr, nullptr);
        return jr::error(ctx, JACC_ERR_INVALID, (std::string("cost model ") + path + ": " + why).c_str());
    }
    if (jr::dry(ctx)) {
        jr::attach_model(ctx, nullptr, nullptr);
        return jr::error(ctx, JACC_ERR_UNSUPPORTED, "the cost model needs the device");
    }
    CostModel *cm = new (std::nothrow) CostModel();
    if (!cm) return JACC_ERR_ALLOC;
    cm->ctx = ctx;
    cm->path = path;
    cm->F = F;
    cm->mu = mu;
    cm->sd = sd;
    int rc = make_nets(ctx, cm, params);
    if (rc) {
        delete cm;
        jr::attach_model(ctx, nullptr, nullptr);
        return rc;
    }
    jr::attach_model(ctx, cm, release_cost_model);
    return JACC_OK;
}

}  // namespace

namespace jr {
bool model_config(jacc_ctx *c, int kind, const int64_t *extent, int ndim, int K, jacc_config *cfg) {
    CostModel *cm = (CostModel *)attached_model(c);
    if (!cm || !stencil_kind(kind, ndim)) return false;
    std::vector<int64_t> sig = {kind, K};
    sig.insert(sig.end(), extent, extent + ndim);
    auto it = cm->cache.find(sig);
    if (it != cm->cache.end()) {
        *cfg = it->second;
        return true;
    }
    if (in_batch(c) || failed(c)) return false;  // no device work while a capture is open
    jacc_candidate best;
    if (pick(c, cm, kind, extent, ndim, &K, 1, true, &best, nullptr, 0, nullptr) != JACC_OK) return false;
    cm->cache[sig] = best.cfg;
    *cfg = best.cfg;
    return true;
}

bool tuned_config(jacc_ctx *c, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args,
                  const double *scalars, int nscalars, jacc_config *cfg) {
    int64_t e[3];
    int ndim = 0, K = 1;
    if (!b || loop_shape(c, kind, nargs, args, e, &ndim, &K) != JACC_OK) return false;
    std::vector<int64_t> sig = {kind, K};
    sig.insert(sig.end(), e, e + ndim);
    for (int d = 0; d < b->ndim && d < 3; ++d) {
        sig.push_back(b->lo[d]);
        sig.push_back(b->hi[d]);
    }
    auto &picks = tuned_picks(c);
    auto it = picks.find(sig);
    if (it != picks.end()) {
        *cfg = it->second;
        return true;
    }
    if (in_batch(c) || failed(c) || dry(c)) return false;
    const std::vector<jacc_candidate> cands = enumerate(kind, e, ndim, &K, 1);
    if (cands.empty()) return false;
    std::vector<double> med(cands.size());
    jacc_tune_opts o{};
    const char *db = tune_db(c);
    o.db_path = (db && *db) ? db : nullptr;
    jacc_candidate best;
    int n = 0;
    if (jacc_tune(c, kind, b, nargs, args, scalars, nscalars, &o, &best, med.data(), (int)med.size(), &n) != JACC_OK)
        return false;
    // the smallest median among candidates that run outside a batch
    // (persistent ones need one), ties to the lowest index
    int bi = -1;
    for (int i = 0; i < n && i < (int)med.size(); ++i)
        if (!cands[(size_t)i].cfg.persistent && (bi < 0 || med[(size_t)i] < med[(size_t)bi])) bi = i;
    if (bi < 0) return false;
    picks[sig] = cands[(size_t)bi].cfg;
    *cfg = cands[(size_t)bi].cfg;
    return true;
}
}  // namespace jr

extern "C" {

int jacc_candidates(int kind, const int64_t *extent, int ndim, const int *ks, int nks, jacc_candidate *out, int cap,
                    int *n) {
    if (!extent || !ks || nks < 1 || nks > 64 || !n || cap < 0 || !stencil_kind(kind, ndim)) return JACC_ERR_INVALID;
    for (int d = 0; d < ndim; ++d)
        if (extent[d] < 3) return JACC_ERR_INVALID;
    for (int q = 0; q < nks; ++q)
        if (ks[q] < 1 || ks[q] > 64) return JACC_ERR_INVALID;
    std::vector<jacc_candidate> c = enumerate(kind, extent, ndim, ks, nks);
    *n = (int)c.size();
    if (out)
        for (int i = 0; i < *n && i < cap; ++i) out[i] = c[i];
    return JACC_OK;
}

int jacc_features(int kind, const int64_t *extent, int ndim, const jacc_candidate *c, float *out) {
    if (!extent || !c || !out || !stencil_kind(kind, ndim)) return JACC_ERR_INVALID;
    for (int d = 0; d < ndim; ++d)
        if (extent[d] < 3) return JACC_ERR_INVALID;
    if (c->K < 1 || c->cfg.bx < 1 || c->cfg.by < 1 || c->cfg.tile < 1 || c->cfg.vec < 1) return JACC_ERR_INVALID;
    features(kind, extent, ndim, *c, out);
    return JACC_OK;
}

const char *jacc_build_key(jacc_ctx *ctx) {
    static thread_local std::string s;
    if (!ctx) return "";
    s = build_key(ctx);
    return s.c_str();
}

double jacc_median(const double *samples, int n) {
    if (!samples || n < 1) return NAN;
    return median_of(std::vector<double>(samples, samples + n));
}

int jacc_argmin(const double *values, int n) {
    if (!values || n < 1) return JACC_ERR_INVALID;
    return argmin_of(values, n);
}

int jacc_tune(jacc_ctx *ctx, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args, const double *scalars,
              int nscalars, const jacc_tune_opts *opts, jacc_candidate *best, double *medians, int cap, int *ncand) {
    if (!ctx || !b || !best || cap < 0 || (cap && !medians)) return JACC_ERR_INVALID;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    if (jr::in_batch(ctx)) return jr::error(ctx, JACC_ERR_INVALID, "tuning inside an open batch");
    try {
        int64_t e[3];
        int ndim = 0, K0 = 1;
        int rc = loop_shape(ctx, kind, nargs, args, e, &ndim, &K0);
        if (rc) return rc;
        const int warmup = opts && opts->warmup > 0 ? opts->warmup : 1;
        const int reps = opts && opts->reps > 0 ? opts->reps : 5;
        std::vector<int> ks;
        if (opts && opts->nks > 0) {
            if (opts->nks > 8) return jr::error(ctx, JACC_ERR_INVALID, "at most 8 partition counts");
            ks.assign(opts->ks, opts->ks + opts->nks);
        } else {
            ks.push_back(K0);
        }
        for (int k : ks)
            if (k < 1 || k > 64) return jr::error(ctx, JACC_ERR_INVALID, "partition counts must lie in [1, 64]");
        const std::vector<jacc_candidate> cands = enumerate(kind, e, ndim, ks.data(), (int)ks.size());
        if (cands.empty()) return jr::error(ctx, JACC_ERR_INVALID, "no candidate fits the loop");
        Db db;
        const char *path = opts ? opts->db_path : nullptr;
        if (path) {
            const std::string why = db_read(path, &db);
            if (!why.empty())
                return jr::error(ctx, JACC_ERR_INVALID, (std::string("timing database ") + path + ": " + why).c_str());
        }
        if (jr::dry(ctx)) return jr::error(ctx, JACC_ERR_UNSUPPORTED, "tuning needs the device");
        auto &sec = db.sections[build_key(ctx)];
        std::vector<double> med(cands.size());
        bool added = false;
        int sweeps = 0;  // per timed graph, set from the first candidate timed
        size_t i = 0;
        while (i < cands.size()) {  // candidates are grouped by K
            const int K = cands[i].K;
            size_t j = i;
            while (j < cands.size() && cands[j].K == K) ++j;
            bool need = false;
            for (size_t q = i; q < j; ++q) need = need || !sec.count(db_key(kind, e, ndim, cands[q]));
            Replica rep;
            jacc_arg targs[2] = {args[0], args[1]};
            if (need) {
                rc = make_replica(ctx, args, K, rep);
                if (rc) return rc;
                targs[0].host = rep.in.data();
                targs[1].host = rep.out.data();
            }
            for (size_t q = i; q < j; ++q) {
                const DbKey k = db_key(kind, e, ndim, cands[q]);
                auto hit = sec.find(k);
                if (hit == sec.end()) {
                    std::vector<double> ms;
                    if (sweeps == 0) {
                        rc = time_candidate(ctx, kind, b, targs, scalars, nscalars, cands[q].cfg, 1, 3, 1, ms);
                        if (rc) return rc;
                        sweeps = sweeps_for(median_of(ms));
                    }
                    rc = time_candidate(ctx, kind, b, targs, scalars, nscalars, cands[q].cfg, warmup, reps, sweeps,
                                        ms);
                    if (rc) return rc;
                    hit = sec.emplace(k, ms).first;
                    added = true;
                }
                med[q] = median_of(hit->second);
            }
            i = j;
        }
        if (path && added && !db_write(path, db))
            return jr::error(ctx, JACC_ERR_INVALID, (std::string("cannot write timing database ") + path).c_str());
        const int bi = argmin_of(med.data(), (int)med.size());
        *best = cands[(size_t)bi];
        for (size_t q = 0; q < med.size() && (int)q < cap; ++q) medians[q] = med[q];
        if (ncand) *ncand = (int)cands.size();
        return JACC_OK;
    } catch (const std::bad_alloc &) {
        return jr::error(ctx, JACC_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return jr::error(ctx, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_model_train(jacc_ctx *ctx, const char *db_path, const char *out_path, const jacc_train_opts *opts,
                     jacc_train_report *report) {
    if (!ctx || !db_path || !out_path) return JACC_ERR_INVALID;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    if (jr::in_batch(ctx)) return jr::error(ctx, JACC_ERR_INVALID, "training inside an open batch");
    if (jr::dry(ctx)) return jr::error(ctx, JACC_ERR_UNSUPPORTED, "the cost model needs the device");
    try {
        const int members = opts && opts->members > 0 ? opts->members : 3;
        const int epochs = opts && opts->epochs > 0 ? opts->epochs : 600;
        const int batch = opts && opts->batch > 0 ? opts->batch : 256;
        const float lr = opts && opts->lr > 0.f ? opts->lr : 1e-3f;
        const uint64_t seed = opts ? opts->seed : 0;
        const int holdout = opts && opts->holdout > 0 ? opts->holdout : 0;
        if (members > 64) return jr::error(ctx, JACC_ERR_INVALID, "at most 64 members");
        Db db;
        const std::string why = db_read(db_path, &db);
        if (!why.empty())
            return jr::error(ctx, JACC_ERR_INVALID, (std::string("timing database ") + db_path + ": " + why).c_str());
        const auto it = db.sections.find(build_key(ctx));
        if (it == db.sections.end() || it->second.empty())
            return jr::error(ctx, JACC_ERR_INVALID, "the timing database holds no rows for this build");
        const int F = JACC_NFEATURES;
        std::vector<float> Xt, yt, Xv, yv;
        std::map<std::vector<int64_t>, int> sig_index;
        for (const auto &kv : it->second) {
            const DbKey &k = kv.first;
            const std::vector<int64_t> sig = {k.kind, k.e[0], k.e[1], k.e[2]};
            auto si = sig_index.emplace(sig, (int)sig_index.size()).first;
            const bool held = holdout > 0 && si->second % holdout == holdout - 1;
            const int ndim = k.e[2] > 0 ? 3 : 2;
            jacc_candidate c{};
            c.cfg.bx = k.bx;
            c.cfg.by = k.by;
            c.cfg.tile = k.tile;
            c.cfg.vec = k.vec;
            c.cfg.persistent = k.pers;
            c.cfg.rows = k.rows;
            c.K = k.K;
            if (!stencil_kind(k.kind, ndim) || k.K < 1 || k.bx < 1 || k.by < 1 || k.tile < 1 || k.vec < 1)
                return jr::error(ctx, JACC_ERR_INVALID, "timing database row of an unknown loop or candidate");
            float f[JACC_NFEATURES];
            features(k.kind, k.e, ndim, c, f);
            const double m = median_of(kv.second);
            if (!(m > 0.0)) continue;
            (held ? Xv : Xt).insert((held ? Xv : Xt).end(), f, f + F);
            (held ? yv : yt).push_back((float)std::log(m));
        }
        const int n = (int)yt.size();
        if (n < 1) return jr::error(ctx, JACC_ERR_INVALID, "no training rows");
        CostModel cm;
        cm.ctx = ctx;
        cm.mu.assign(F, 0.f);
        cm.sd.assign(F, 1.f);
        for (int f = 0; f < F; ++f) {
            double s = 0.0, s2 = 0.0;
            for (int i = 0; i < n; ++i) s += Xt[(size_t)i * F + f];
            const double mean = s / n;
            for (int i = 0; i < n; ++i) {
                const double d = Xt[(size_t)i * F + f] - mean;
                s2 += d * d;
            }
            const double sd = std::sqrt(s2 / n);
            cm.mu[f] = (float)mean;
            cm.sd[f] = sd > 0.0 ? (float)sd : 1.f;
        }
        std::vector<std::vector<float>> params;
        for (int q = 0; q < members; ++q) params.push_back(init_params(F, seed * 1000003ull + (uint64_t)q));
        int rc = make_nets(ctx, &cm, params);
        if (rc) return rc;
        std::vector<float> loss((size_t)epochs);
        for (int q = 0; q < members; ++q) {
            rc = jacc_model_fit(cm.nets[q], Xt.data(), yt.data(), n, epochs, batch, lr, seed + 1 + (uint64_t)q,
                                q == 0 ? loss.data() : nullptr);
            if (rc) return rc;
            rc = jacc_model_get_params(cm.nets[q], params[q].data(), (int)params[q].size());
            if (rc) return rc;
        }
        float mse = 0.f;
        if (!yv.empty()) {
            std::vector<float> yh;
            rc = predict(&cm, Xv, (int)yv.size(), yh);
            if (rc) return rc;
            double acc = 0.0;
            for (size_t i = 0; i < yv.size(); ++i) acc += (double)(yh[i] - yv[i]) * (yh[i] - yv[i]);
            mse = (float)(acc / (double)yv.size());
        }
        if (!write_model_file(out_path, build_key(ctx), F, cm.mu, cm.sd, params))
            return jr::error(ctx, JACC_ERR_INVALID, (std::string("cannot write ") + out_path).c_str());
        if (report) {
            report->rows = n;
            report->signatures = (int)sig_index.size();
            report->loss_first = loss[0];
            report->loss_last = loss[(size_t)epochs - 1];
            report->heldout_mse = mse;
        }
        return JACC_OK;
    } catch (const std::bad_alloc &) {
        return jr::error(ctx, JACC_ERR_ALLOC, "host allocation failed");
    } catch (...) {
        return jr::error(ctx, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_model_load(jacc_ctx *ctx, const char *path) {
    if (!ctx || !path) return JACC_ERR_INVALID;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    if (jr::in_batch(ctx)) return jr::error(ctx, JACC_ERR_INVALID, "loading a model inside an open batch");
    try {
        return load_model(ctx, path);
    } catch (...) {
        return jr::error(ctx, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_model_unload(jacc_ctx *ctx) {
    if (!ctx) return JACC_ERR_INVALID;
    if (jr::in_batch(ctx)) return jr::error(ctx, JACC_ERR_INVALID, "unloading a model inside an open batch");
    jr::attach_model(ctx, nullptr, nullptr);
    return JACC_OK;
}

int jacc_model_pick(jacc_ctx *ctx, int kind, const int64_t *extent, int ndim, const int *ks, int nks,
                    jacc_candidate *best, float *pred, int cap, int *ncand) {
    if (!ctx || !extent || !ks || nks < 1 || nks > 64 || !best || cap < 0 || (cap && !pred)) return JACC_ERR_INVALID;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    if (jr::in_batch(ctx)) return jr::error(ctx, JACC_ERR_INVALID, "model inference inside an open batch");
    CostModel *cm = (CostModel *)jr::attached_model(ctx);
    if (!cm) return jr::error(ctx, JACC_ERR_INVALID, "no cost model is attached");
    if (!stencil_kind(kind, ndim)) return jr::error(ctx, JACC_ERR_UNSUPPORTED, "picks cover JACOBI2D and HEAT3D");
    for (int d = 0; d < ndim; ++d)
        if (extent[d] < 3) return jr::error(ctx, JACC_ERR_INVALID, "extents below 3");
    for (int q = 0; q < nks; ++q)
        if (ks[q] < 1 || ks[q] > 64) return jr::error(ctx, JACC_ERR_INVALID, "partition counts must lie in [1, 64]");
    try {
        return pick(ctx, cm, kind, extent, ndim, ks, nks, false, best, pred, cap, ncand);
    } catch (...) {
        return jr::error(ctx, JACC_ERR_INVALID, "internal error");
    }
}

int jacc_choose(jacc_ctx *ctx, int kind, const jacc_bounds *b, int nargs, const jacc_arg *args, const double *scalars,
                int nscalars, const char *model_path, const jacc_tune_opts *opts, jacc_candidate *out, int *source) {
    if (!ctx || !out || !source) return JACC_ERR_INVALID;
    if (jr::failed(ctx)) return JACC_ERR_DEVICE;
    try {
        int64_t e[3];
        int ndim = 0, K0 = 1;
        int rc = loop_shape(ctx, kind, nargs, args, e, &ndim, &K0);
        if (rc) return rc;
        std::string reasons;
        if (model_path) {
            CostModel *cm = (CostModel *)jr::attached_model(ctx);
            rc = (cm && cm->path == model_path) ? JACC_OK : jacc_model_load(ctx, model_path);
            if (!rc) {
                std::vector<int> ks;
                if (opts && opts->nks > 0)
                    ks.assign(opts->ks, opts->ks + std::min(opts->nks, 8));
                else
                    ks.push_back(K0);
                rc = jacc_model_pick(ctx, kind, e, ndim, ks.data(), (int)ks.size(), out, nullptr, 0, nullptr);
                if (!rc) {
                    *source = JACC_CHOICE_MODEL;
                    return JACC_OK;
                }
            }
            reasons = std::string("model: ") + jacc_last_error(ctx);
            if (jr::failed(ctx)) return JACC_ERR_DEVICE;
        }
        if (opts) {
            rc = jacc_tune(ctx, kind, b, nargs, args, scalars, nscalars, opts, out, nullptr, 0, nullptr);
            if (!rc) {
                *source = JACC_CHOICE_TUNER;
                if (!reasons.empty()) jr::error(ctx, JACC_OK, reasons.c_str());
                return JACC_OK;
            }
            reasons += (reasons.empty() ? "" : "; ") + std::string("tuner: ") + jacc_last_error(ctx);
            if (jr::failed(ctx)) return JACC_ERR_DEVICE;
        }
        *out = jacc_candidate{};
        out->K = K0;
        *source = JACC_CHOICE_DEFAULT;
        if (!reasons.empty()) jr::error(ctx, JACC_OK, reasons.c_str());
        return JACC_OK;
    } catch (...) {
        return jr::error(ctx, JACC_ERR_INVALID, "internal error");
    }
}

}  // extern "C"
