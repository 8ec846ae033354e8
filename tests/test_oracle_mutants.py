"""Planted mistakes in the oracle must fail its pins.

Each mutant is a copy of the oracle's C source with one plausible mistake (a flipped
sign, a dropped normalisation, a wrong index or representative, an off-by-one median,
a strict instead of inclusive comparison, a wrong transpose, a wrong constant).  It is
compiled on the CPU and the pin suite is run against it in a subprocess; the suite
must fail for every mutant.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mr1l_oracle.c")

MUTANTS = {
    "dft_sign": ("sw[r] = (ld)sign * sinl(ang);", "sw[r] = -(ld)sign * sinl(ang);"),
    "dft_no_normalisation": ("y[2 * q] = (double)(re / (ld)Ml);", "y[2 * q] = (double)(re);"),
    "floor_mod_representative": ("if (r < 0) r += m;", "if (r < 0) r = -r;"),
    "hash_drops_first_dim": ("for (int32_t u = 0; u < d; ++u)\n        acc += (__int128)k",
                             "for (int32_t u = 1; u < d; ++u)\n        acc += (__int128)k"),
    "median_off_by_one": ("if (L & 1) return v[L / 2];", "if (L & 1) return v[L / 2 + 1 < L ? L / 2 + 1 : 0];"),
    "vote_strict": ("if (v[i] >= vote_min) {", "if (v[i] > vote_min) {"),
    "singleton_test": ("if (cnt[off[l] + hh[q * L + l]] == 1) {", "if (cnt[off[l] + hh[q * L + l]] <= 2) {"),
    "sort_ascending": ("if (x->key > y->key) return -1;\n    if (x->key < y->key) return 1;",
                       "if (x->key < y->key) return -1;\n    if (x->key > y->key) return 1;"),
    "sample_phase_sign": ("ld ang = TWO_PI_L * frac;", "ld ang = -TWO_PI_L * frac;"),
    "adjoint_not_transposed": ("re += a * c - b * sn;\n                im += a * sn + b * c;",
                               "re += a * c + b * sn;\n                im += -a * sn + b * c;"),
    "anchor_index": ("(uint64_t)anchor[u - t]);\n        aph[i] = acc;", "(uint64_t)anchor[0]);\n        aph[i] = acc;"),
    "splitmix_shift": ("x ^= x >> 27;", "x ^= x >> 26;"),
    "eq42_factor": ("double bound = 0.25 *", "double bound = 0.5 *"),
    "bucket_sum_conjugate": ("acc[2 * h + 1] += (ld)coef[2 * i + 1];", "acc[2 * h + 1] -= (ld)coef[2 * i + 1];"),
    "threshold_not_squared": ("return m2 >= theta * theta;", "return m2 >= theta;"),
    "driver_range": ("I1[(int64_t)(t - 1) * K + a] = a - N;", "I1[(int64_t)(t - 1) * K + a] = a - N + 1;"),
    "step1_threshold": ("if (m2 >= theta * theta) { keys[nk].m2", "if (m2 < theta * theta) { keys[nk].m2"),
    "step1_coordinate": ("pf[q] = poly_freq[(int64_t)(t - 1) * s_poly + q];", "pf[q] = poly_freq[(int64_t)t % d * s_poly + q];"),
    "median_weight_even": ("wq[2 * vs[L / 2].l + part] = 1.0;", "wq[2 * vs[0].l + part] = 1.0;"),
    "mask_32_bits": ("mask |= 1ull << l;", "mask |= 1u << (l & 31);"),
    "bspline_sign": ("s += ((j & 1) ? -binom : binom) * pw;", "s += binom * pw;"),
    "bspline_norm_power": ("for (int32_t e = 0; e < 2 * m; ++e) p *= sc;", "for (int32_t e = 0; e < m; ++e) p *= sc;"),
    "bspline_scale": ("return bspline_norm_const(m) * (ld)m * trunc_power_bspline(m, (ld)m * x);",
                      "return bspline_norm_const(m) * trunc_power_bspline(m, (ld)m * x);"),
    "bspline_anchor": ("else x = (ld)anchor[u - t] / 4294967296.0L;", "else x = (ld)anchor[0] / 4294967296.0L;"),
    "pfpn_pfn_threshold": ("(med > 1.0 ? 2 : 0)", "(med >= 1.0 ? 2 : 0)"),
    "pfpn_pfp_threshold": ("(med > 0.0 ? 1 : 0)", "(med > 0.5 ? 1 : 0)"),
    "pfpn_alone": ("M[l])] == 1;\n        if", "M[l])] <= 2;\n        if"),
    "pfpn_support_counted": ("for (int64_t i = 0; i < n_active; ++i)\n            cnt[",
                             "for (int64_t i = 0; i <= n_active; ++i)\n            cnt["),
    "pfpn_detected_set": ("if (i >= n_active && !(cls[i] & 1)) continue;", "if (!(cls[i] & 1)) continue;"),
}


def _run_mutant(name, workdir):
    """Compile one mutant and run the pin suite against it -> (return code, output tail)."""
    old, new = MUTANTS[name]
    src = open(SRC).read()
    if src.count(old) != 1:
        return None, f"mutation site not unique/found: {name}"
    d = os.path.join(workdir, name)
    os.makedirs(d, exist_ok=True)
    msrc = os.path.join(d, "mutant.c")
    with open(msrc, "w") as fh:
        fh.write(src.replace(old, new))
    mlib = os.path.join(d, "libmutant.so")
    oracle.build_from(msrc, mlib)
    env = dict(os.environ, MR1L_ORACLE_LIB=mlib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_results(tmp_path_factory):
    """Every mutant's pin run, several at a time (each is its own process)."""
    workdir = str(tmp_path_factory.mktemp("mutants"))
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {name: ex.submit(_run_mutant, name, workdir) for name in sorted(MUTANTS)}
        return {name: f.result() for name, f in futs.items()}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, mutant_results):
    rc, out = mutant_results[name]
    assert rc is not None, out
    assert rc != 0, f"mutant {name} survived the pins:\n{out}"
