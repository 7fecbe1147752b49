"""The pins are strong enough: each test here plants one plausible mistake in
a copy of the oracle's C source (a dropped term, a wrong sign, index or
comparison, a transposed operand), builds it, and runs the pin suite against
it; at least one pin must fail.  Only copies are changed; oracle.c is read."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PIN_FILES = [os.path.join(ROOT, "tests", f)
             for f in ("test_oracle_pins.py", "test_oracle_containment.py", "test_oracle_filters.py",
                       "test_oracle_strands.py", "test_oracle_abundance.py")]

# (name, original text, planted mistake); each original occurs exactly once.
MUTANTS = [
    ("code of T", "case 'T': case 't': return 3;", "case 'T': case 't': return 2;"),
    ("N k-mers seed", "if (c == 4) ok = 0;", "if (c == 5) ok = 0;"),
    ("k-mer base order", "v = v * 4 + (c & 3);", "v = v + ((uint64_t)(c & 3) << (2 * t));"),
    ("hash drops a step", "return z ^ (z >> 31);", "return z;"),
    ("hash shift", "z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;", "z = (z ^ (z >> 28)) * 0x94d049bb133111ebULL;"),
    ("rightmost tie", "if (best < 0 || h[i] < h[best]) best = i;", "if (best < 0 || h[i] <= h[best]) best = i;"),
    ("short sequence", "int64_t win = nk < w ? nk : w;", "int64_t win = w;"),
    ("window one short", "for (int64_t i = s; i < s + win; i++) {", "for (int64_t i = s; i < s + win - 1; i++) {"),
    ("diagonal sign", "hit[nh].diag = (int64_t)ix->occ[o].pos - mpos[i];",
     "hit[nh].diag = mpos[i] - (int64_t)ix->occ[o].pos;"),
    ("max_occ inclusive", "if (ix->max_occ > 0 && hi - lo > (int64_t)ix->max_occ) continue;",
     "if (ix->max_occ > 0 && hi - lo >= (int64_t)ix->max_occ) continue;"),
    ("strict min_hits", "if ((uint64_t)(j - i) >= min_hits) {", "if ((uint64_t)(j - i) > min_hits) {"),
    ("hits ascending", "if (p->hits != q->hits) return p->hits > q->hits ? -1 : 1;",
     "if (p->hits != q->hits) return p->hits < q->hits ? -1 : 1;"),
    ("genome tie descending",
     "if (p->genome != q->genome) return p->genome < q->genome ? -1 : 1;\n    if (p->diag != q->diag) return p->diag < q->diag ? -1 : 1;\n    if (p->strand != q->strand) return p->strand < q->strand ? -1 : 1;\n    return 0;\n}\n\n/* O15",
     "if (p->genome != q->genome) return p->genome > q->genome ? -1 : 1;\n    if (p->diag != q->diag) return p->diag < q->diag ? -1 : 1;\n    if (p->strand != q->strand) return p->strand < q->strand ? -1 : 1;\n    return 0;\n}\n\n/* O15"),
    ("strand tie reverse first", "if (p->strand != q->strand) return p->strand < q->strand ? -1 : 1;\n    return 0;\n}\n\n/* O15",
     "if (p->strand != q->strand) return p->strand > q->strand ? -1 : 1;\n    return 0;\n}\n\n/* O15"),
    ("reverse without complement", "out[j] = c == 4 ? 4 : (uint8_t)(3 - c);", "out[j] = c;"),
    ("complement without reverse", "uint8_t c = q[m - 1 - j];", "uint8_t c = q[j];"),
    ("strands merged in counting", "hit[j].strand == hit[i].strand)", "1)"),
    ("strand-1 filter on the read", "filter_codes(kind, oriented[cand[c].strand], m,", "filter_codes(kind, oriented[0], m,"),
    ("abundance ignores unique evidence",
     "counts[set[i]] += U ? (uint64_t)(((unsigned __int128)unique[set[i]] << 32) / U)\n                                    : ((uint64_t)1 << 32) / nt;",
     "counts[set[i]] += ((uint64_t)1 << 32) / nt;"),
    ("abundance cutoff strict", "int keep = C > 0 && (unsigned __int128)counts[t] * den >= C * num;\n        if (keep)",
     "int keep = C > 0 && (unsigned __int128)counts[t] * den > C * num;\n        if (keep)"),
    ("multi reads counted as unique", "if (nt == 1) unique[set[0]]++;", "unique[set[0]]++;"),
    ("abundance over all taxa", "if (keep) { K += counts[t]; kept++; }", "K += counts[t]; if (keep) kept++;"),
    ("abundance rounded twice", "abund[t] = keep ? div_nearest(counts[t], K) : 0.0;",
     "abund[t] = keep ? (double)counts[t] / (double)(uint64_t)K : 0.0;"),
    ("top_n off by one", "if (top_n > 0 && nc > (int64_t)top_n) nc = top_n;",
     "if (top_n > 0 && nc > (int64_t)top_n + 1) nc = top_n + 1;"),
    ("N is a fifth letter", "    if (qc == 4) return 1;\n    if (p < 0 || p >= glen) return 1;\n    uint8_t rc = gcode[p];\n    if (rc == 4) return 1;",
     "    if (p < 0 || p >= glen) return 1;\n    uint8_t rc = gcode[p];"),
    ("outside genome matches", "if (p < 0 || p >= glen) return 1;", "if (p < 0 || p >= glen) return 0;"),
    ("band one row short", "int64_t rows = 2 * (int64_t)E + 1;", "int64_t rows = 2 * (int64_t)E;"),
    ("no skip after obstacle", "        c += 1;\n        if (c > E) break;\n        j += 1;",
     "        c += 1;\n        if (c > E) break;"),
    ("early stop", "        c += 1;\n        if (c > E) break;", "        c += 1;\n        if (c >= E) break;"),
    ("cap at E", "return c < E + 1 ? c : E + 1;", "return c < E ? c : E;"),
    ("strict accept", "out->accept[c] = (uint8_t)(a <= E);", "out->accept[c] = (uint8_t)(a < E);"),
    ("E rounds down", "if (e_mode == 1) return (int)((num + 999) / 1000);", "if (e_mode == 1) return (int)(num / 1000);"),
    ("worst accepted count", "if (a <= E && (best < 0 || a < best)) best = a;",
     "if (a <= E && (best < 0 || a > best)) best = a;"),
    ("multi counted once", "if (ntax > 1) res->multi_reads[t]++;", "if (ntax > 1 && t == only) res->multi_reads[t]++;"),
    ("unique ignores ties", "if (ntax == 1) res->unique_reads[only]++;", "if (ntax >= 1) res->unique_reads[only]++;"),
    ("containment counts a key once", "for (int64_t o = lo; o < hi; o++) local[ix->occ[o].genome] += 1;",
     "if (hi > lo) local[ix->occ[lo].genome] += 1;"),
    ("containment cap inclusive", "if (ix->max_occ && (uint64_t)(hi - lo) > ix->max_occ) continue;",
     "if (ix->max_occ && (uint64_t)(hi - lo) >= ix->max_occ) continue;"),
    ("selection not strict", "> (unsigned __int128)M * num) selected", ">= (unsigned __int128)M * num) selected"),
    ("selection in 64 bits", "if ((unsigned __int128)hits[g] * den > (unsigned __int128)M * num)",
     "if (hits[g] * den > M * num)"),
    ("hamming off row 0", "for (int64_t j = 0; j < m; j++) c += obstacle(q[j], gcode, glen, diag + j);",
     "for (int64_t j = 0; j < m; j++) c += obstacle(q[j], gcode, glen, diag + j + 1);"),
    ("base count rounds down", "int64_t v = (l1 + 1) / 2;", "int64_t v = l1 / 2;"),
    ("base count counts outside", "if (p >= 0 && p < glen && gcode[p] < 4) nw[gcode[p]]++;",
     "if (p >= 0 && p < glen && gcode[p] < 4) nw[gcode[p]]++; else nw[0]++;"),
    ("filter kinds swapped", "case 1: return hamming_codes(", "case 1: return base_count_codes("),
    ("q-gram window without the band", "for (int64_t p = diag - E; p + QGRAM_Q <= diag + m + E; p++) {",
     "for (int64_t p = diag; p + QGRAM_Q <= diag + m; p++) {"),
    ("q-gram rounds down", "int64_t val = (missing + QGRAM_Q - 1) / QGRAM_Q;", "int64_t val = missing / QGRAM_Q;"),
    ("q-gram window N shared", "if (x < 0 || x >= glen || gcode[x] == 4) ok = 0;", "if (x < 0 || x >= glen) ok = 0;"),
    ("SHD amends runs of three", "int amend = j > 0 && k < m && k - j <= 2;", "int amend = j > 0 && k < m && k - j <= 3;"),
    ("SHD amends at the read ends", "int amend = j > 0 && k < m && k - j <= 2;", "int amend = k - j <= 2;"),
    ("SHD band one row short", "for (int64_t d = -(int64_t)E; d <= E; d++) {", "for (int64_t d = -(int64_t)E; d < E; d++) {"),
]


def _run_pins(lib: str, stop_at_first: bool):
    """The pin suite against the oracle library at `lib`, in a process of its own
    (one oracle thread: several of these run at once)."""
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    args = [sys.executable, "-m", "pytest", *PIN_FILES, "-q", "-p", "no:cacheprovider"] + (["-x"] if stop_at_first else [])
    return subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def mutant_runs(tmp_path_factory):
    """Every mutant built and run against the pins, several at a time: name ->
    (occurrences of its site in oracle.c, return code of the pin suite)."""
    from concurrent.futures import ThreadPoolExecutor
    base = tmp_path_factory.mktemp("mutants")
    src = open(SRC).read()

    def one(i_m):
        i, (name, orig, mut) = i_m
        sites = src.count(orig)
        if sites != 1:
            return name, (sites, None)
        d = base / f"m{i}"
        d.mkdir()
        mutant_c = d / "oracle_mutant.c"
        mutant_c.write_text(src.replace(orig, mut))
        lib = str(d / "liboracle_mutant.so")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", lib, str(mutant_c),
                               "-lm"])
        return name, (sites, _run_pins(lib, True).returncode)

    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        return dict(ex.map(one, enumerate(MUTANTS)))


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, orig, mut, mutant_runs):
    sites, rc = mutant_runs[name]
    assert sites == 1, f"mutation site of '{name}' not found exactly once"
    assert rc != 0, f"no pin caught the planted mistake '{name}'"


def test_unmutated_copy_passes_the_pins(tmp_path):
    lib = str(tmp_path / "liboracle_copy.so")
    oracle.build(lib)
    r = _run_pins(lib, False)
    assert r.returncode == 0, r.stdout[-2000:]
