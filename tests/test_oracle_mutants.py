"""The pins must be able to fail: each case plants one plausible mistake (a dropped term,
a wrong sign, a wrong index or operand) into a temporary copy of the oracle's C source,
builds it, and checks that the pin suite rejects the mutant.  Nothing here touches the
committed oracle or the GPU."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ranky_oracle.c")

MUTANTS = {
    "gram_drops_diagonal": ("for (int64_t k2 = k1; k2 <", "for (int64_t k2 = k1 + 1; k2 <"),
    "rotation_angle_sign": ("double zeta = (beta - alpha) / (2.0 * gamma);",
                            "double zeta = (alpha - beta) / (2.0 * gamma);"),
    "eig_new_diagonal_sign": ("C[5 * i + 3] = a - t * g;", "C[5 * i + 3] = a + t * g;"),
    "hestenes_u_rotation_sign": ("U[(size_t)row * m + p] = cs * x - sn * y;",
                                 "U[(size_t)row * m + p] = cs * x + sn * y;"),
    "backproject_no_division": ("acc = acc / sigma[i];", "acc = acc * sigma[i];"),
    "backproject_wrong_sigma_index": ("acc = acc / sigma[i];", "acc = acc / sigma[0];"),
    "sign_rule_inverted": ("double sgn = (W[(size_t)best * n + c] < 0.0) ? -1.0 : 1.0;",
                           "double sgn = (W[(size_t)best * n + c] < 0.0) ? 1.0 : -1.0;"),
    "occupancy_single_counts_empty": ("if (cnt[(size_t)b * M + m] == 1) single[b] += 1;",
                                      "if (cnt[(size_t)b * M + m] == 0) single[b] += 1;"),
    "block_bounds_drop_remainder": ("start[b] = ((int64_t)b * N) / D;", "start[b] = (int64_t)b * (N / D);"),
    "proxy_without_sigma": ("Pm[(size_t)r * pcap + pcols] = Ub[(size_t)r * n + i] * sb[i];",
                            "Pm[(size_t)r * pcap + pcols] = Ub[(size_t)r * n + i];"),
    "householder_wrong_shift": ("v[0] -= alpha;", "v[0] += alpha;"),
    "empty_row_vector_missing": ("U[(size_t)empty[i - n] * k + i] = 1.0;",
                                 "U[(size_t)empty[i - n] * k + i] = 0.0;"),
    "gram_route_forgets_sqrt": ("s[a] = sqrt(lam > 0.0 ? lam : 0.0);", "s[a] = (lam > 0.0 ? lam : 0.0);"),
    "threshold_without_sqrt": ("double tau = fmax(tol, sqrt((double)n * u_gram)) * s1;",
                               "double tau = fmax(tol, (double)n * u_gram) * s1;"),
    "stale_row_in_two_sided_update": ("gq[c] = sn * x + cs * y;", "gq[c] = sn * x + cs * gq[c] * 0.0;"),
    "bf16_truncates_instead_of_rounding": ("const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;",
                                           "const uint32_t r = u & 0xffff0000u;"),
    "bf16_ties_away_from_even": ("const uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;",
                                 "const uint32_t r = (u + 0x8000u) & 0xffff0000u;"),
    "split_product_drops_cross_term": ("G[(size_t)a * nr + b] += h1 * h2 + h1 * l2 + l1 * h2;",
                                       "G[(size_t)a * nr + b] += h1 * h2 + h1 * l2;"),
    "checker_inserts_two": ("vals_out[pos] = 1.0;", "vals_out[pos] = 2.0;"),
    "checker_no_fallback": ("ins[nins++] = (neigh_col >= 0 ? neigh_col : rand_col) * M + m;",
                            "if (neigh_col >= 0) ins[nins++] = neigh_col * M + m;"),
    "checker_neighbour_columns_of_next_block": ("if (n2 >= c0 && n2 < c1 && !mark[n2 - c0]) {",
                                                "if (n2 >= c1 && n2 < c1 + w && !mark[n2 - c1]) {"),
    "split_product_keeps_lo_lo": ("G[(size_t)a * nr + b] += h1 * h2 + h1 * l2 + l1 * h2;",
                                  "G[(size_t)a * nr + b] += h1 * h2 + h1 * l2 + l1 * h2 + l1 * l2;"),
}


def _build_and_run(name, old, new, workdir):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutant {name}: pattern not found"
    mdir = os.path.join(workdir, name)
    os.makedirs(mdir, exist_ok=True)
    csrc = os.path.join(mdir, "mutant.c")
    with open(csrc, "w") as f:
        f.write(src.replace(old, new, 1))
    so = os.path.join(mdir, "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", so, csrc, "-lm"])
    env = dict(os.environ, RANKY_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, p.returncode, p.stdout[-400:]


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda kv: _build_and_run(kv[0], kv[1][0], kv[1][1], str(tmp_path)),
                              MUTANTS.items()))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, "mutants not caught by the pins: " + ", ".join(n for n, _ in survivors)
