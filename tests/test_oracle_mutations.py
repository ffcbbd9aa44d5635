"""The oracle's pins must catch plausible mistakes: each case plants one
mistake into a scratch copy of the oracle (C or Python), rebuilds it and runs
tests/test_oracle_pins.py against it, which must fail. CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (file inside oracle/, original text, planted mistake); the first occurrence is changed
MUTATIONS = [
    ("nbvh_oracle.c", "return (uint32_t)(v[0] + r1 * (v[1] + r1 * v[2]));",
     "return (uint32_t)(v[1] + r1 * (v[0] + r1 * v[2]));"),                       # transposed dense stride
    ("nbvh_oracle.c", "wk *= bit ? w[a] : (1.0 - w[a]);", "wk *= bit ? (1.0 - w[a]) : w[a];"),  # swapped weights
    ("nbvh_oracle.c", "float frac = ((float)s + 0.5f)", "float frac = ((float)s + 0.0f)"),    # stratum offset
    ("nbvh_oracle.c", "double bce = (z0 > 0.0 ? z0 : 0.0) - z0 * h", "double bce = (z0 > 0.0 ? z0 : 0.0) + z0 * h"),
    ("nbvh_oracle.c", "if (k > 0) acc = pre[(k - 1) * width + j] > 0.0 ? acc : 0.0;",
     "if (k > 1) acc = pre[(k - 1) * width + j] > 0.0 ? acc : 0.0;"),             # ReLU derivative
    ("nbvh_oracle.c", "double mh = m[i] / c1, vh = v[i] / c2;", "double mh = m[i], vh = v[i] / c2;"),  # bias correction
    ("nbvh_oracle.c", "tn = fmaxf(tn, ta);", "tn = fmaxf(tn, tb);"),                # slab operand
    ("nbvh_oracle.c", "u[s * L * F + l * F + f] = acc;", "u[l * c->n_samples * F + s * F + f] = acc;"),  # concatenation
    ("nbvh_oracle.c", "if (t < best) {", "if (t <= best) {"),                      # tie rule
    ("nbvh_oracle.c", "g[1] = h * w_t * oc_sgn(st - tau) * st * (1.0 - st) / B;",
     "g[1] = h * w_t * oc_sgn(st - tau) * st / B;"),                              # sigmoid derivative
    ("nbvh_oracle.c", "((uint32_t)v[1] * 2654435761u)", "((uint32_t)v[1] * 2654435769u)"),  # hash prime
    ("nbvh_oracle.c", "float rel = p - c->scene_lo[a];", "float rel = p + c->scene_lo[a];"),  # normalisation sign
    ("nbvh_oracle.c", "        id |= OC_INSIDE_TAG;\n", "\n"),                       # inside chord left untagged
    ("nbvh_oracle.c", "t = b - tau * (b - a);", "t = a + tau * (b - a);"),           # reversed distance from the entry
    ("nbvh_oracle.c", "if (!(t > (double)ray_tmin[r])) continue;", ""),            # hits behind the origin kept
    ("__init__.py", "out[inside, 4:7] = -out[inside, 4:7]", "out[inside, 4:7] = out[inside, 4:7]"),  # direction not reversed
    ("nbvh_oracle.c", "double d = 2.0 * (ah - a) / den;",
     "double d = (2.0 * (ah - a) * den - (ah - a) * (ah - a) * 2.0 * ah) / (den * den);"),  # albedo denominator differentiated
    ("nbvh_oracle.c", "r[i] = 2.0 * log(q) + log(p);", "r[i] = log(q) + log(p);"),  # rank: q not squared
    ("nbvh_oracle.c", "exp(r[i] - rmax)", "exp(rmax - r[i])"),                     # acceptance order inverted
    ("nbvh_oracle.c", "for (int j = 0; j < H * width; ++j) m =", "for (int j = width; j < H * width; ++j) m ="),  # kink scan skips layer 0
]


def _run_pins(tmp):
    env = dict(os.environ, PYTHONPATH=str(tmp))
    return subprocess.run([sys.executable, "-m", "pytest", os.path.join(str(tmp), "tests", "test_oracle_pins.py"),
                           "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                          cwd=str(tmp), env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("fname,orig,planted", MUTATIONS, ids=[str(i) for i in range(len(MUTATIONS))])
def test_pins_catch_planted_mistake(tmp_path, fname, orig, planted):
    for d in ("oracle", "nbvh_synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("__pycache__", "_nbvh_oracle.so*", "test_oracle_mutations.py"))
    path = tmp_path / "oracle" / fname
    src = path.read_text()
    assert orig in src, "mutation anchor not found: %r" % orig
    path.write_text(src.replace(orig, planted, 1))  # the first occurrence only
    res = _run_pins(tmp_path)
    assert res.returncode != 0, "planted mistake survived the pins: %r -> %r" % (orig, planted)
