// Autotuner of the filter step: entry points that time the filter variants of
// each pair bucket on a caller's reads, select per bucket, and save / load
// the selection as JSON keyed by the GPU architecture.
#include <cstdio>
#include <fstream>
#include <sstream>

#include "classify.hpp"

namespace mt {

// pair_read[c] = r for every candidate c of read r.
__global__ void k_expand_pairs(const u64 *__restrict__ cand_off, u64 n, u32 *__restrict__ pair_read) {
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    for (u64 c = cand_off[r]; c < cand_off[r + 1]; c++) pair_read[c] = (u32)r;
}

static std::string device_arch() {
    int dev = 0;
    MT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    MT_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

// The quoted strings of a JSON text, in order (our own flat format only).
static std::vector<std::string> json_strings(const std::string &t) {
    std::vector<std::string> out;
    for (size_t i = 0; i < t.size(); i++) {
        if (t[i] != '"') continue;
        std::string s;
        size_t j = i + 1;
        for (; j < t.size() && t[j] != '"'; j++) {
            if (t[j] == '\\' && j + 1 < t.size()) j++;
            s += t[j];
        }
        MT_REQUIRE(j < t.size(), "unterminated string in tuning file");
        out.push_back(s);
        i = j;
    }
    return out;
}

}  // namespace mt

using mt::guarded;

extern "C" int mt_tune_buckets(uint32_t *n) {
    if (!n) return MT_EINVAL;
    *n = (uint32_t)mt::tune_buckets();
    return MT_OK;
}

extern "C" int mt_tune_info(uint32_t bucket, mt_tune_bucket *out) {
    if (!out) {
        mt::set_last_error("mt_tune_info: null argument");
        return MT_EINVAL;
    }
    return guarded("mt_tune_info", [&] { mt::tune_info((int)bucket, *out); });
}

extern "C" int mt_tune_set(uint32_t bucket, uint32_t variant) {
    return guarded("mt_tune_set", [&] { mt::tune_set((int)bucket, (int)variant); });
}

extern "C" int mt_tune_reset(void) {
    return guarded("mt_tune_reset", [&] { mt::tune_reset(); });
}

extern "C" int mt_autotune(const mt_index *index, const mt_query_params *params, const mt_seqs *reads, uint32_t reps,
                           void *stream) {
    if (!index || !params || !reads) {
        mt::set_last_error("mt_autotune: null argument");
        return MT_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    return guarded("mt_autotune", [&] {
        using namespace mt;
        validate_query(*params);
        MT_REQUIRE(reads->n == 0 || (reads->seq && reads->offsets), "null read arrays");
        const u64 n = reads->n;
        CallScope scope(s);
        mt_result res;
        mt_result_init(res, n, index->n_taxa, s);
        ReadBatch rb;
        rb.prepare(*reads, params->e_mode, params->e_value, s);
        MT_HIP(hipMemcpyAsync(res.read_E.p, rb.read_E.p, (n ? n : 1) * sizeof(u16), hipMemcpyDeviceToDevice, s));
        Timer tm;
        tm.stream = s;
        classify_per_stage(*index, *params, *reads, rb, res, tm, s);
        u32 f = 0;
        read_back(s, rb.flags.p, &f, sizeof f);
        check_flags(f);
        u64 nc = 0;
        read_back(s, res.cand_off.p + n, &nc, sizeof nc);
        if (nc == 0) return;
        DBuf<u32> pair_read(nc);
        DBuf<u16> approx(nc);
        DBuf<u8> accept(nc);
        k_expand_pairs<<<grid_for(n, 256), 256, 0, s>>>(res.cand_off.p, n, pair_read.p);
        MT_HIP(hipGetLastError());
        FilterArgs fa{};
        fa.pair_read = pair_read.p;
        fa.pair_genome = res.genome.p;
        fa.pair_diag = res.diag.p;
        fa.pair_E = nullptr;
        fa.read_E = res.read_E.p;
        fa.n_dev = nullptr;
        fa.n_host = nc;
        fa.n_reads = n;
        fa.read_off = reads->offsets;
        fa.read_blk = rb.planes.blk_off.p;
        fa.read_lohi = rb.planes.lohi.p;
        fa.read_nb = rb.planes.nb.p;
        fa.n_genomes = index->n_genomes;
        fa.meta = index->meta.p;
        fa.ref_lohi = index->ref.lohi.p;
        fa.ref_nb = index->ref.nb.p;
        fa.approx = approx.p;
        fa.accept = accept.p;
        fa.flags = rb.flags.p;
        autotune_filter(fa, nc, reps, s);
        read_back(s, rb.flags.p, &f, sizeof f);
        check_flags(f);
    });
}

extern "C" int mt_tune_save(const char *path) {
    if (!path) {
        mt::set_last_error("mt_tune_save: null path");
        return MT_EINVAL;
    }
    return guarded("mt_tune_save", [&] {
        std::ostringstream o;
        o << "{\"arch\": \"" << mt::device_arch() << "\", \"buckets\": {";
        for (int b = 0; b < mt::tune_buckets(); b++) {
            mt_tune_bucket tb;
            mt::tune_info(b, tb);
            o << (b ? ", " : "") << "\"" << tb.name << "\": \"" << tb.variant_names[tb.current] << "\"";
        }
        o << "}}\n";
        std::ofstream f(path);
        MT_REQUIRE(f.good(), std::string("cannot write ") + path);
        f << o.str();
        MT_REQUIRE(f.good(), std::string("cannot write ") + path);
    });
}

extern "C" int mt_tune_load(const char *path) {
    if (!path) {
        mt::set_last_error("mt_tune_load: null path");
        return MT_EINVAL;
    }
    return guarded("mt_tune_load", [&] {
        std::ifstream f(path);
        MT_REQUIRE(f.good(), std::string("cannot read ") + path);
        std::stringstream ss;
        ss << f.rdbuf();
        const std::vector<std::string> t = mt::json_strings(ss.str());
        MT_REQUIRE(t.size() >= 3 && t[0] == "arch" && t[2] == "buckets" && (t.size() - 3) % 2 == 0,
                   "not a tuning file");
        MT_REQUIRE(t[1] == mt::device_arch(), "tuning file was made for " + t[1]);
        // validate every entry before changing anything
        std::vector<std::pair<int, int>> sel;
        for (size_t i = 3; i < t.size(); i += 2) {
            int found = -1, var = -1;
            for (int b = 0; b < mt::tune_buckets(); b++) {
                mt_tune_bucket tb;
                mt::tune_info(b, tb);
                if (t[i] != tb.name) continue;
                found = b;
                for (uint32_t v = 0; v < tb.n_variants; v++)
                    if (t[i + 1] == tb.variant_names[v]) var = (int)v;
            }
            MT_REQUIRE(found >= 0, "unknown bucket " + t[i]);
            MT_REQUIRE(var >= 0, "unknown variant " + t[i + 1] + " for " + t[i]);
            sel.emplace_back(found, var);
        }
        for (auto &bv : sel) mt::tune_set(bv.first, bv.second);
    });
}
