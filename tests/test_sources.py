"""Static checks of the device sources.

Every word of heap metadata (object bitmaps, block type words, pins and the
block-state bitmaps) is read and written only through agent-scope atomic
operations: the eight XCDs of the chip have L2 caches of their own, so a
plain load can hit a line that an XCD's L2 still holds from before another
XCD's atomics changed it (a stale object-bitmap snapshot makes a do-all visit
and delete slots that are no longer live).  This scans the sources for
element accesses of those arrays by plain indexing."""
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = sorted(glob.glob(os.path.join(ROOT, "paper_1809_07444_amd", "csrc", "*.hip")) +
                 glob.glob(os.path.join(ROOT, "paper_1809_07444_amd", "csrc", "*.hpp")))
META = ["obj_bitmap", "block_type", "pins", "bitmaps", "units"]


def strip_comments(text):
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.sub(r"//[^\n]*", "", text)


def test_sources_found():
    assert any(p.endswith("dsoar_device.hpp") for p in SOURCES)


def test_heap_metadata_is_never_indexed_plainly():
    bad = []
    for path in SOURCES:
        text = strip_comments(open(path).read())
        for name in META:
            for m in re.finditer(r"\b(?:\w+\s*(?:\.|->)\s*)?" + name + r"\s*\[", text):
                line = text.count("\n", 0, m.start()) + 1
                bad.append(f"{os.path.basename(path)}:{line}: {m.group(0)}")
    assert bad == []
