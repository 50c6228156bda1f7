"""Host-side check of the build: every registration function the library
calls (glbm_internal.h: GLBM_OBJECTS for glbm_inst.hip, GLBM_OBJECTS3 for
glbm_inst3.hip) is defined by exactly one object of build.tasks(), with the
defines that select it, so the link cannot miss or duplicate a kernel set."""
import os
import re

from paper_1905_04597_amd import build

HEADER = os.path.join(build.CSRC, "glbm_internal.h")


def _macro(name):
    text = open(HEADER).read()
    m = re.search(r"#define %s\(X\)(.*?)\n(?!\s)" % name, text.replace("\\\n", " "), re.S)
    assert m, name
    return m.group(1)


def _defines(task):
    return {k: int(v) for k, v in (d[2:].split("=") for d in task[2])}


def _kind(d):
    """Registration kind (glbm_inst.hip's GLBM_KIND) of an object's defines."""
    if not d["GLBM_COMPACT"]:
        return 0
    if d.get("GLBM_WALLS", 0) and 1 <= d["GLBM_LEVEL"] <= 7:
        return 2
    return 1


def test_every_registration_has_one_object():
    objs = [t for t in build.tasks() if t[0].endswith("glbm_inst.hip")]
    have = {}
    for t in objs:
        d = _defines(t)
        key = (d["GLBM_EVEN"], _kind(d), d["GLBM_LEVEL"])
        assert key not in have, (key, t[1], have.get(key))
        have[key] = t[1]
    want = {tuple(int(v) for v in m) for m in re.findall(r"X\((\d+), (\d+), (\d+)\)", _macro("GLBM_OBJECTS"))}
    assert want == set(have), (sorted(want - set(have)), sorted(set(have) - want))


def test_every_3d_part_has_one_object():
    parts = [_defines(t)["GLBM_3D_PART"] for t in build.tasks() if t[0].endswith("glbm_inst3.hip")]
    want = [int(k) for k in re.findall(r"X\((\d+)\)", _macro("GLBM_OBJECTS3"))]
    assert sorted(parts) == sorted(want) and len(set(parts)) == len(parts)
    src = open(os.path.join(build.CSRC, "glbm_inst3.hip")).read()
    for k in want:
        assert "GLBM_3D_PART == %d" % k in src and "register3_%d()" % k in src


def test_object_names_are_distinct():
    names = [t[1] for t in build.tasks()]
    assert len(names) == len(set(names))
