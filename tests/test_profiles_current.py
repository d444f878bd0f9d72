"""The committed rocprofv3 summaries were taken on the kernels in this tree:
each records the hash of the kernel sources it was measured on, and that
hash must be the current one (a kernel change without a new profile fails
here, rather than leaving figures that describe other code)."""
import glob
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_profile_is_of_the_current_kernels():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt")))
    assert files, "no profiles"
    current = bench.kernel_source_hash()
    for f in files:
        text = open(f).read()
        m = re.search(r"kernel_source_hash:\s*([0-9a-f]{16})", text)
        assert m, "%s records no kernel_source_hash" % os.path.basename(f)
        assert m.group(1) == current, (os.path.basename(f), m.group(1), current)


def test_every_profile_names_its_command():
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        text = open(f).read()
        assert "rocprofv3" in text and "bench.py" in text, os.path.basename(f)
