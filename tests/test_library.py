"""CPU checks of the C-ABI library: it is built, loads, and exports every
entry point declared in include/galpic.h (no compute calls, no GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "galpic.h")
LIB = os.path.join(ROOT, "paper_1608_00215_amd", "libgalpic.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_step_calls():
    names = declared_functions()
    for call in ("gp_init_grid", "gp_set_v_gal", "gp_deposit", "gp_fft_fwd",
                 "gp_galilean_psatd_update", "gp_fft_inv", "gp_gather_push"):
        assert call in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_match_header():
    from paper_1608_00215_amd import galpic

    assert sorted(galpic.EXPORTS) == declared_functions()


def test_field_selector_order_matches_header():
    from paper_1608_00215_amd import galpic

    text = open(HEADER).read()
    body = text[text.index("GP_EX = 0"):text.index("GP_N_FIELDS")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = [n.strip().split("=")[0].strip() for n in body.split(",") if n.strip()]
    assert [n[3:] for n in names] == galpic.FIELDS


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1608_00215_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", src.replace("no fallback", "")) or \
                    "import oracle" not in src, f
                assert "import oracle" not in src and "from oracle" not in src, f


PASSAGES = ("the transformed equations", "the update display", "the deposition paragraph",
            "the simulation parameters")
CITED_CALLS = ("gp_init_grid", "gp_set_v_gal", "gp_bind_particles", "gp_deposit",
               "gp_fft_fwd", "gp_galilean_psatd_update", "gp_fft_inv", "gp_gather_push",
               "gp_gather_push_deposit", "gp_step", "gp_run", "gp_step_graph",
               "gp_half_push", "gp_field_ptr")


def test_hot_path_calls_cite_a_passage():
    """Every call of the step (and the field accessor) names, in the comment
    just above its declaration, the passage of the paper that defines it,
    from the list of passages the header's preamble explains."""
    text = open(HEADER).read()
    preamble = text[:text.index("#ifndef GALPIC_H")]
    for p in PASSAGES:
        assert f'"{p}"' in preamble, p
    for call in CITED_CALLS:
        m = re.search(r"/\*((?:(?!\*/).)*)\*/\s*(?:gp_status\s+[a-z_0-9]+\([^;]*;\s*)*gp_status\s+"
                      + call + r"\(", text, flags=re.S)
        assert m, call
        comment = " ".join(re.sub(r"\n\s*\*", " ", m.group(1)).split())
        assert "Paper:" in comment, call
        cited = comment[comment.index("Paper:"):]
        assert any(p in cited for p in PASSAGES), (call, cited[:80])


def test_field_pointer_accessor_declared():
    assert "gp_field_ptr" in declared_functions()
    text = open(HEADER).read()
    assert re.search(r"gp_status\s+gp_field_ptr\(gp_ctx \*ctx, int run, int which, void \*\*dev_ptr\)",
                     text)
