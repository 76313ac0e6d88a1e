"""__graft_entry__.build() works from a tree that holds no built library.

The source tree is copied without any compiled artefact (no libmrs.so, no
oracle library, no object files); build() must compile both libraries there
and leave a package whose entry points are bound to the new libmrs.so.  No
GPU is needed: hipcc cross-compiles for gfx950.
"""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# what build() compiles and imports: the package, the oracle, the C header,
# the input generators and the entry module (sources only)
SOURCE_ROOTS = ("paper_2604_12083_amd", "oracle", "include", "synth", "__graft_entry__.py")
SKIP_DIRS = {"_build", "__pycache__"}
SKIP_EXT = (".so", ".o", ".a", ".pyc", ".log")


def _copy_sources(dst):
    os.makedirs(dst, exist_ok=True)
    for top in SOURCE_ROOTS:
        src = os.path.join(ROOT, top)
        if os.path.isfile(src):
            shutil.copy2(src, os.path.join(dst, top))
            continue
        for dirpath, dirnames, filenames in os.walk(src):
            dirnames[:] = [d for d in dirnames if d not in SKIP_DIRS and not d.startswith(".")]
            rel = os.path.relpath(dirpath, ROOT)
            os.makedirs(os.path.join(dst, rel), exist_ok=True)
            for f in filenames:
                if f.endswith(SKIP_EXT) or ".so.tmp" in f:
                    continue
                shutil.copy2(os.path.join(dirpath, f), os.path.join(dst, rel, f))


def test_build_from_clean_tree(tmp_path):
    dst = str(tmp_path / "tree")
    _copy_sources(dst)
    assert not os.path.exists(os.path.join(dst, "paper_2604_12083_amd", "libmrs.so"))
    code = ("import __graft_entry__ as g; g.build(); import paper_2604_12083_amd as m; "
            "assert m.library_loaded(); print(m.LIB_PATH)")
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1")
    out = subprocess.run([sys.executable, "-c", code], cwd=dst, env=env, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    lib = os.path.join(dst, "paper_2604_12083_amd", "libmrs.so")
    assert out.stdout.strip().splitlines()[-1] == lib
    assert os.path.exists(lib) and os.path.exists(os.path.join(dst, "oracle", "liboracle.so"))


def test_package_without_library_raises_on_use(tmp_path):
    """Without libmrs.so the package imports (the build module needs it) and
    every entry point fails loudly instead of falling back to anything."""
    dst = str(tmp_path / "tree")
    _copy_sources(dst)
    code = ("import paper_2604_12083_amd as m\n"
            "assert not m.library_loaded()\n"
            "try:\n    m.mrs_context_create(0)\nexcept ImportError as e:\n    print('raised', e)\n"
            "else:\n    raise SystemExit('no error')\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=dst, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "raised" in out.stdout and "libmrs.so is missing" in out.stdout
