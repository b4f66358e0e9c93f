"""The product path and the oracle are independent: nothing in the package or
the C ABI names, imports or links the oracle or its library, loading the
package maps no oracle code (nor the seeded input generators, which only the
autotuner's command line uses for the batched table's shapes), and the package
fails loudly (no fallback) when its HIP library is missing."""
import os
import re
import subprocess
import sys

from paper_2003_09133_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2003_09133_amd")
PRODUCT_DIRS = (PKG, os.path.join(ROOT, "include"))
SOURCE_EXT = (".py", ".cpp", ".hip", ".h", ".txt")


def product_sources():
    for top in PRODUCT_DIRS:
        for dirpath, dirnames, files in os.walk(top):
            dirnames[:] = [d for d in dirnames if not d.startswith(("_build", "__pycache__"))]
            for f in files:
                if f.endswith(SOURCE_EXT):
                    yield os.path.join(dirpath, f)


def test_product_sources_never_name_the_oracle():
    pattern = re.compile(r"oracle", re.IGNORECASE)
    hits = []
    for path in product_sources():
        for i, line in enumerate(open(path, encoding="utf-8", errors="replace"), 1):
            if pattern.search(line):
                hits.append(f"{os.path.relpath(path, ROOT)}:{i}: {line.strip()}")
    assert not hits, "\n".join(hits)


def test_library_links_and_exports_nothing_of_the_oracle():
    needed = subprocess.run(["readelf", "-d", _abi.LIB_PATH], capture_output=True, text=True, check=True).stdout
    libs = re.findall(r"\(NEEDED\)\s+Shared library: \[([^\]]+)\]", needed)
    assert libs, needed
    assert not [l for l in libs if "oracle" in l or "lfsynth" in l], libs
    syms = subprocess.run(["nm", "-D", _abi.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert not [l for l in syms.splitlines() if "oracle" in l or "lfsynth" in l]


def test_loading_the_package_maps_no_oracle_code():
    probe = ("import sys; sys.path.insert(0, %r); import paper_2003_09133_amd as lf; lf._abi.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "print('modules', sorted(m for m in sys.modules if m.startswith(('oracle', 'lfsynth')))); "
             "print('mapped', sorted({l.split()[-1] for l in maps.splitlines() "
             "if 'oracle' in l or 'lfsynth' in l}))" % ROOT)
    out = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, cwd="/", check=True).stdout
    assert "modules []" in out and "mapped []" in out, out


def test_missing_library_fails_loudly():
    probe = ("import sys; sys.path.insert(0, %r); import paper_2003_09133_amd as lf\n"
             "try:\n    lf.default_config((15, 15, 3, 3, 3))\nexcept ImportError as e:\n    print('raised', e)\n"
             "else:\n    print('no error')" % ROOT)
    env = dict(os.environ, LFBP_LIB=os.path.join(ROOT, "_no_such_dir_", "liblfbp.so"))
    out = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, cwd="/", env=env,
                         check=True).stdout
    assert out.startswith("raised liblfbp.so not found"), out
