"""The oracle's pins must catch plausible mistakes.

Each mutant is a copy of oracle.c with one planted mistake (a dropped term, a wrong comparison,
a wrong index, a wrong rounding ...), compiled on the CPU into a temporary library. The pin
suites are run against it in a subprocess and at least one pin must fail.
"""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTANTS = {
    "channel_threshold_not_strict": ("af > t_channel * nz[s]", "af >= t_channel * nz[s]"),
    "seed_threshold_not_strict": ("af > t_seed * nz[s]", "af >= t_seed * nz[s]"),
    "seed_uses_channel_threshold": ("af > t_seed * nz[s]", "af > t_channel * nz[s]"),
    "cluster_threshold_strict": ("(float)q_raw >= t_cluster * sqrtf(sum_n2)",
                                 "(float)q_raw > t_cluster * sqrtf(sum_n2)"),
    "noise_not_squared": ("sum_n2 = fmaf(nz[i], nz[i], sum_n2);", "sum_n2 += nz[i];"),
    "no_sqrt": ("t_cluster * sqrtf(sum_n2)", "t_cluster * sum_n2"),
    "noise_sum_rounds_product": ("sum_n2 = fmaf(nz[i], nz[i], sum_n2);",
                                 "sum_n2 = sum_n2 + nz[i] * nz[i];"),
    "noise_sum_right_to_left": ("sum_n2 = fmaf(nz[i], nz[i], sum_n2);",
                                "sum_n2 = fmaf(nz[r + l - i], nz[r + l - i], sum_n2);"),
    "threshold_in_double": ("(float)q_raw >= t_cluster * sqrtf(sum_n2)",
                            "(double)q_raw >= (double)t_cluster * sqrt((double)sum_n2)"),
    "gain_wrong_apv": ("rintf((float)a[i] / g[i / NAPV])", "rintf((float)a[i] / g[0])"),
    "gain_multiplies": ("rintf((float)a[i] / g[i / NAPV])", "rintf((float)a[i] * g[i / NAPV])"),
    "gain_truncates": ("rintf((float)a[i] / g[i / NAPV])", "truncf((float)a[i] / g[i / NAPV])"),
    "bary_no_half": ("((double)i + 0.5)", "((double)i)"),
    "seedless_runs_kept": ("if (!has_seed) continue;", ""),
    "bad_flag_ignored": ("if (bad != 0) return 1;", ""),
    "negative_noise_ok": ("isnan(n) || n < 0.0f || isinf(n)", "isnan(n) || isinf(n)"),
    "zero_gain_ok": ("isnan(g) || g <= 0.0f", "isnan(g) || g < 0.0f"),
    "bary_fallback_wrong": ("(float)l + (float)width * 0.5f", "(float)l"),
    "U2_dropped": ("if (count == 0) return 1;", ""),
    "U3_off_by_one": ("if (first + count > NSTRIP) return 1;", "if (first + count >= NSTRIP) return 1;"),
    "U4_dropped": ("if (first < next_free) return 1;", ""),
    "U5_truncation_dropped": ("if (q + 2 + count > len) return 1;", "if (q + 2 + count > len) break;"),
    "length_big_endian": ("plen = (uint32_t)fed[pos] | ((uint32_t)fed[pos + 1] << 8);",
                          "plen = ((uint32_t)fed[pos] << 8) | (uint32_t)fed[pos + 1];"),
    "U1_keeps_later_channels": ("for (; ch < NCH; ++ch) {", "for (; ch < ch; ++ch) {"),
    "trailing_ignored": ("for (ch = 0; ch < NCH; ++ch) chan_status[(uint64_t)f * NCH + ch] |= ORACLE_FED_TRAILING;", ""),
    "apv_index_half_channel": ("float gs = g[s / NAPV];", "float gs = g[0];"),
}


# Planted mistakes in the module-aware function (readings M1-M4), killed by its own pins.
MODULE_MUTANTS = {
    "rows_ignore_joins": ("while (c1 < n_ch && c1 % NCH != 0 && joins[c1]) ++c1;",
                          "while (0) ++c1;"),
    "rows_cross_feds": ("while (c1 < n_ch && c1 % NCH != 0 && joins[c1]) ++c1;",
                        "while (c1 < n_ch && joins[c1]) ++c1;"),
    "bary_from_row_start": ("num += ((double)(i - ch_off) + 0.5) * (double)cq;",
                            "num += ((double)i + 0.5) * (double)cq;"),
    "record_channel_row_start": ("o->channel = (uint32_t)(c0 + l / NSTRIP);",
                                 "o->channel = (uint32_t)c0;"),
    "first_in_row_numbering": ("o->first = (uint16_t)(l % NSTRIP);", "o->first = (uint16_t)l;"),
    "gain_of_row_start": ("float q = rintf((float)adc[base + i] / gain[(base + i) / NAPV]);",
                          "float q = rintf((float)adc[base + i] / gain[(base + l) / NAPV]);"),
}
MARK = "/* Module-aware clustering."


def _mutate(src, old, new, module):
    """Applies the mutation inside the plain functions (before MARK) or inside the module-aware
    one (after it); the site must be unique there."""
    head, tail = src.split(MARK, 1)
    part = tail if module else head
    assert part.count(old) == 1, f"mutation site not unique/found: {old!r}"
    part = part.replace(old, new)
    return (head + MARK + part) if module else (part + MARK + tail)


@pytest.mark.parametrize("name", sorted(MUTANTS) + sorted(MODULE_MUTANTS))
def test_mutant_is_killed(name, tmp_path):
    module = name in MODULE_MUTANTS
    old, new = (MODULE_MUTANTS if module else MUTANTS)[name]
    src = open(oracle.SRC).read()
    msrc = tmp_path / "oracle_mutant.c"
    msrc.write_text(_mutate(src, old, new, module))
    lib = str(tmp_path / "liboracle_mutant.so")
    oracle.build(force=True, src=str(msrc), out=lib)
    env = dict(os.environ, ORACLE_LIB=lib, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu",
                        *([os.path.join(HERE, "test_oracle_modules.py")] if module else
                          [os.path.join(HERE, "test_oracle_unpack.py"),
                           os.path.join(HERE, "test_oracle_cluster.py")])],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived every pin:\n{r.stdout[-2000:]}"
