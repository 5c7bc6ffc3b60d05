"""The design notes point at files and tests that exist: every test module,
test function and profile summary that the design doc cites is in the tree."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _design():
    with open(os.path.join(ROOT, "DESIGN.md")) as fh:
        return fh.read()


def _test_defs():
    defs = set()
    for f in os.listdir(os.path.join(ROOT, "tests")):
        if f.endswith(".py"):
            with open(os.path.join(ROOT, "tests", f)) as fh:
                defs.update(re.findall(r"^def (test_\w+)", fh.read(), re.M))
    return defs


def test_cited_test_modules_and_functions_exist():
    s = _design()
    mods = set(re.findall(r"(test_\w+\.py)", s))
    assert mods, "the design notes cite their tests"
    for m in mods:
        assert os.path.exists(os.path.join(ROOT, "tests", m)), m
    defs = _test_defs()
    for f in set(re.findall(r"`(test_\w+)`", s)):
        assert f in defs, f


def test_cited_profiles_exist():
    s = _design()
    cited = set(re.findall(r"profiles/([\w.]+\.(?:md|json|txt))", s))
    cited |= set(re.findall(r"`(\w+\.(?:md|json))`", s)) & set(os.listdir(os.path.join(ROOT, "profiles")))
    assert cited
    for p in cited:
        assert os.path.exists(os.path.join(ROOT, "profiles", p)), p
