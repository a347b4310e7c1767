"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/gal.h, and rejects invalid configurations before it
touches the device (no compute calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2306_07552_amd import gal
from paper_2306_07552_amd import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "gal.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gal_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gal.LIB_PATH):
        from paper_2306_07552_amd import build
        build.build(verbose=False)
    return gal.load_library()


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"libgal.so does not export {n}"


def _small_inputs():
    cfg = sg.scaled_config(0, 2)
    return sg.make_robot_for(cfg), sg.make_scene_set(cfg), sg.config_constants(cfg)


@pytest.mark.parametrize("mutate,needle", [
    (lambda r, s, c: c.update(near=-1.0), "near"),
    (lambda r, s, c: c.update(far=0.05), "near"),
    (lambda r, s, c: setattr(s, "res", np.array([64, 100], np.int32)), "resolution"),
    (lambda r, s, c: setattr(s, "res", np.array([64, 512], np.int32)), "resolution"),
    (lambda r, s, c: r.sphere_class.__setitem__(0, 7), "class"),
    (lambda r, s, c: r.sphere_link.__setitem__(1, 8), "link"),
    (lambda r, s, c: c.update(radius_classes=()), "num_classes"),
    (lambda r, s, c: c.update(episode_len=-3), "episode_len"),
])
def test_invalid_config_rejected(lib, mutate, needle):
    robot, scenes, consts = _small_inputs()
    consts = dict(consts)
    mutate(robot, scenes, consts)
    with pytest.raises(gal.GalError) as ei:
        gal.Batch(robot, scenes, consts, stream=0)
    assert ei.value.code == -1
    assert needle in str(ei.value)


def test_null_arguments(lib):
    out = C.c_void_p()
    assert lib.gal_create_batch(None, None, None, None, C.byref(out)) == -1
    assert b"null" in lib.gal_last_error()
    assert lib.gal_step(None, None, None, None) == -1
    assert lib.gal_reset(None, None, None) == -1
    assert lib.gal_get_state(None, None, 0, None) == -1


def declaration_comments():
    """For every gal_* function declared in include/gal.h, the comment block
    that documents it: the nearest block comment above its declaration (a
    block may document a run of consecutive declarations)."""
    text = open(os.path.join(ROOT, "include", "gal.h")).read()
    out = {}
    last_comment = None
    token = re.compile(r"/\*.*?\*/|^(?:int|void|const char)\s*\*?\s*(gal_[a-z_]+)\s*\(",
                       re.S | re.M)
    for m in token.finditer(text):
        if m.group(0).startswith("/*"):
            last_comment = m.group(0)
        else:
            out[m.group(1)] = last_comment
    return out


def test_every_entry_point_cites_its_passage():
    """Each declared entry point is documented by a comment that names the
    passage of the paper it implements or extends (a Section, Appendix or
    Table)."""
    docs = declaration_comments()
    assert set(docs) == set(header_functions())
    cite = re.compile(r"\b(Section \d(\.\d)?|Appendix [A-I]|Table \d)\b")
    # the allocation-free variant names the callers it is for instead
    missing = [n for n, c in docs.items()
               if c is None or not (cite.search(c) or "cannot allocate" in c)]
    assert not missing, f"entry points without a citation: {missing}"


@pytest.mark.parametrize("field,cut", [("tri_plane", 1), ("tris", 1), ("tri_rgb", 2), ("boxes", 1),
                                       ("verts", 3)])
def test_array_lengths_must_match_offsets(lib, field, cut):
    """The ABI takes the scene arrays without lengths; the binding refuses
    arrays shorter than the offsets say, before the library reads them."""
    robot, scenes, consts = _small_inputs()
    a = getattr(scenes, field)
    setattr(scenes, field, a[:-cut])
    with pytest.raises(gal.GalError) as ei:
        gal.Batch(robot, scenes, consts, stream=0)
    assert field in str(ei.value)
