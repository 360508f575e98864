"""The pins catch plausible mistakes: each case below plants one mistake in
a copy of the oracle's C source (a dropped or doubled term, a wrong
comparison, a swapped rounding, a missing step), builds it, and runs the
oracle's pin tests against it; at least one pin must fail. The unmodified
copy must pass them all."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = [os.path.join(HERE, f) for f in ("test_oracle.py", "test_oracle_ot.py",
                                        "test_oracle_costs.py", "test_oracle_ot_clustered.py")]

# (name, text in oracle.c, replacement, every occurrence?)
MUTATIONS = [
    ("admissible without the +1",
     "return (int64_t)cost_of(c, b, a) + 1 == (int64_t)y_a[a] + (int64_t)y_b[b];",
     "return (int64_t)cost_of(c, b, a) == (int64_t)y_a[a] + (int64_t)y_b[b];", False),
    ("highest proposer wins",
     "if (proposer[a] < 0 || b < proposer[a]) proposer[a] = b;",
     "if (proposer[a] < 0 || b > proposer[a]) proposer[a] = b;", False),
    ("losers skip a column", "pos[i] += 1;", "pos[i] += 2;", False),
    ("y(a) falls by two", "if (taken_by[a] >= 0) y_a[a] -= 1;",
     "if (taken_by[a] >= 0) y_a[a] -= 2;", False),
    ("y(b) rises by two", "if (!won[i]) y_b[B_prime[i]] += 1;",
     "if (!won[i]) y_b[B_prime[i]] += 2;", False),
    ("stop test strict", "if (n_i <= T) break;", "if (n_i < T) break;", False),
    ("no completion", "if (complete && status == ORC_OK) {\n        int64_t ia = 0;",
     "if (0) {\n        int64_t ia = 0;", False),
    ("eq. (1) rounds up",
     "if (!(c >= 0.0 && c <= 1.0)) return ORC_E_RANGE;\n            k[b * ldk + a] = (int16_t)floor(c / eps);",
     "if (!(c >= 0.0 && c <= 1.0)) return ORC_E_RANGE;\n            k[b * ldk + a] = (int16_t)ceil(c / eps);",
     False),
    ("distance not squared", "s = fmaf(t, t, s);", "s = s + fabsf(t);", True),
    ("cost not scaled by the maximum",
     "double c = (double)d2[b * n_a + a] / (double)m;", "double c = (double)d2[b * n_a + a];",
     False),
    ("Euclidean without the root", "double c = sqrt((double)d2[b * n_a + a] / (double)m);",
     "double c = (double)d2[b * n_a + a] / (double)m;", False),
    ("images not normalised", "dst[w][i * d + j] = src[w][i * d + j] / sum;",
     "dst[w][i * d + j] = src[w][i * d + j];", False),
    ("image cost not halved", "double c = (double)t * 0.5;", "double c = (double)t;", False),
    ("no free-copy raise", "y_b[b] = group_max[cs->row_pt[b]];", "(void)0;", False),
    ("supplies rounded up", "int64_t v = (int64_t)floor(th * nu[b]);",
     "int64_t v = (int64_t)ceil(th * nu[b]);", False),
    ("excess not returned", "plan[b * n_a + a] = v - take;", "plan[b * n_a + a] = v;", False),
    ("point costs without the matrix not scaled by the maximum",
     "double v = (double)sq_f32(c->X + r * c->d, c->Y + q * c->d, c->d) / (double)c->m;",
     "double v = (double)sq_f32(c->X + r * c->d, c->Y + q * c->d, c->d);", False),
    ("clusters: evictions from the lower level's slot",
     "int32_t p = Z[a] & 1;\n            if (Z[a] == 0) {",
     "int32_t p = (Z[a] - 1) & 1;\n            if (Z[a] == 0) {", False),
    ("clusters: new pairs at the top level",
     "int32_t q = (Z[a] - 1) & 1;", "int32_t q = Z[a] & 1;", False),
    ("clusters: Z kept when the top runs out", "if (cap[a] == 0) Z[a] -= 1;", "(void)0;", False),
    ("clusters: copies left over rise by two", "if (want[b] > 0) Y[b] += 1;",
     "if (want[b] > 0) Y[b] += 2;", False),
    ("clusters: evicted copies lost", "F[b] = want[b] + evicted[b];", "F[b] = want[b];", False),
    ("clusters: free demand copies not first",
     "int64_t u = taken < G[a] ? taken : G[a];", "int64_t u = 0;", False),
    ("clusters: proposers served in descending b",
     "            /* (ii) each point serves its proposers in ascending b */\n            for (int64_t b = 0; b < n_b; ++b) {",
     "            /* (ii) each point serves its proposers in ascending b */\n            for (int64_t b = n_b - 1; b >= 0; --b) {",
     False),
    ("clusters: completion dropped", "if (flow) flow[b * n_a + a] += v;", "(void)0;", False),
    ("point costs without the matrix transposed",
     "sq_f32(c->X + r * c->d, c->Y + q * c->d, c->d)",
     "sq_f32(c->X + q * c->d, c->Y + r * c->d, c->d)", False),
]


def _build(tmp_path, name, src):
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-I", os.path.join(ROOT, "oracle"), "-o", str(so), str(c), "-lm"],
                   check=True, cwd=os.path.join(ROOT, "oracle"))
    return str(so)


def _run_pins(lib):
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unmodified_copy_passes_the_pins(tmp_path):
    rc, out = _run_pins(_build(tmp_path, "same", open(SRC).read()))
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new,every", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, every):
    src = open(SRC).read()
    count = src.count(old)
    assert count >= 1 and (every or count == 1), f"{name}: pattern found {count} times"
    mutant = src.replace(old, new) if every else src.replace(old, new, 1)
    rc, out = _run_pins(_build(tmp_path, "mutant", mutant))
    assert rc != 0, f"no pin caught: {name}\n{out}"
