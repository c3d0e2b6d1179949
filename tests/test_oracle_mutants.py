"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source (a
dropped term, a wrong sign, a wrong index, a transposed operand), builds it
into a temporary library and runs the pin tests against it in a subprocess:
the pins must fail.  Nothing here touches the GPU.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "orc.c")

MUTANTS = {
    "kernel_transposed": ("s += wr[v] * xr[v];",
                          "s += w[(((long)co * Cin + ci) * k + v) * k + u] * xr[v];"),
    "bias_dropped": ("s += bias_full ? bias[((long)co * f1 + t1) * f2 + t2] : bias[co];", ""),
    "relu_sign": ("double a = (relu && s < 0.0) ? 0.0 : s;", "double a = (relu && s > 0.0) ? 0.0 : s;"),
    "crop_off_by_one": ("if (t1 >= r && t1 < r + n1 && t2 >= r && t2 < r + n2)\n          out[((long)co * n1 + (t1 - r)) * n2 + (t2 - r)] = a;",
                        "if (t1 >= r - 1 && t1 < r - 1 + n1 && t2 >= r && t2 < r + n2)\n          out[((long)co * n1 + (t1 - r + 1)) * n2 + (t2 - r)] = a;"),
    "fc_transposed": ("for (int m = 0; m < M; ++m) s += wfc[(long)p * M + m] * y[(long)b * M + m];",
                      "for (int m = 0; m < M; ++m) s += wfc[(long)m * N + p] * y[(long)b * M + m];"),
    "measure_transposed": ("for (int n = 0; n < N; ++n) s += phi[(long)m * N + n] * x[(long)b * N + n];",
                           "for (int n = 0; n < N; ++n) s += phi[(long)n * M + m] * x[(long)b * N + n];"),
    "loss_grad_scale": ("g[p] = 2.0 * d / B;", "g[p] = 2.0 * d;"),
    "relu_mask_dropped": ("gz[t] = (relu && !(z[l][t] > 0.0)) ? 0.0 : gv;", "gz[t] = gv;"),
    "dgrad_index": ("int t1 = i + (k - 1) - u, t2 = j + (k - 1) - v;", "int t1 = i + u, t2 = j + (k - 1) - v;"),
    "adam_no_bias_correction": ("double mh = m[q] / c1, vh = v[q] / c2;", "double mh = m[q], vh = v[q] / c2;"),
    "psnr_peak": ("if (x[p] > peak) peak = x[p];", ""),
    "noise_scale": ("const double s = ne > 0.0 ? sqrt(ny / ne) * pow(10.0, -snr_db / 20.0) : 0.0;",
                    "const double s = ne > 0.0 ? sqrt(ny / ne) * pow(10.0, -snr_db / 10.0) : 0.0;"),
    "dct_sign": ("C[(long)k * n + i] = a * cos(pi * (2 * i + 1) * k / (2.0 * n));",
                 "C[(long)k * n + i] = a * cos(pi * (2 * i - 1) * k / (2.0 * n));"),
    "round_ties_away": ("if (d > 0.5 || (d == 0.5 && fmod(fl, 2.0) != 0.0)) fl += 1.0;", "if (d >= 0.5) fl += 1.0;"),
    "round_no_subnormals": ("int E = e - 1 < emin ? emin : e - 1;\n  double q = ldexp(1.0, E - p + 1);",
                            "int E = e - 1;\n  double q = ldexp(1.0, E - p + 1);"),
    "e4m3_max": ("return round_format(v, 4, -6, 448.0, 1);", "return round_format(v, 4, -6, 480.0, 1);"),
    "bf16_bits": ("return round_format(v, 8, -126, BF16_MAX, 0);", "return round_format(v, 7, -126, BF16_MAX, 0);"),
    "proxy_not_rounded": ("double v = q_value(a[0][p], qs->xt);", "double v = a[0][p];"),
    "hidden_not_rounded": ("double v = q_value(a[l + 1][i], qs->a[l]);", "double v = a[l + 1][i];"),
    "y_not_rounded": ("for (int m = 0; m < M; ++m) yq[m] = q_value(yb[m], qs->y);",
                      "for (int m = 0; m < M; ++m) yq[m] = yb[m];"),
    "errmodel_weight_term": ("wc[l][i] = q_var(w[l][i], qs->w[l]) + ca * w2[l][i];", "wc[l][i] = ca * w2[l][i];"),
    "errmodel_relu_mask": ("Vn[i] = (relu && !(a[l + 1][i] > 0.0)) ? 0.0 : t1[i] + t2[i];",
                           "Vn[i] = t1[i] + t2[i];"),
    "errmodel_acc_coeff": ("return acc_fp32 ? (double)n / 24.0 * ldexp(1.0, -46) : 0.0;",
                           "return acc_fp32 ? (double)n / 24.0 * ldexp(1.0, -48) : 0.0;"),
}


def _build_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = os.path.join(tmp, f"orc_{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmp, f"liborc_{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                           "-ffp-contract=off", "-I", os.path.join(ROOT, "oracle"), "-o", so, path, "-lm"])
    return so


def _pins_fail(so):
    env = dict(os.environ, ORC_LIB_PATH=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_grad.py"),
                        os.path.join(ROOT, "tests", "test_oracle_quant.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode != 0, r.stdout[-400:]


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        sos = {n: _build_mutant(n, tmp) for n in MUTANTS}
        with ThreadPoolExecutor(max_workers=4) as ex:
            res = dict(zip(sos, ex.map(_pins_fail, sos.values())))
    survivors = [n for n, (failed, _) in res.items() if not failed]
    assert not survivors, f"pins did not catch: {survivors}"


def test_unmutated_copy_passes():
    """Control: the same harness on an unmodified copy passes (so failures above are the mutation's)."""
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "liborc_control.so")
        subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", so, SRC, "-lm"])
        failed, out = _pins_fail(so)
        assert not failed, out
