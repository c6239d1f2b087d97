"""Readers for the worked-example fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_sections(name):
    """Parse 'key = value' lines, optionally grouped under [section] headers."""
    sections, cur = {}, {}
    sections[""] = cur
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = {}
                sections[line[1:-1]] = cur
                continue
            k, v = line.split("=", 1)
            cur[k.strip()] = v.strip()
    return sections
