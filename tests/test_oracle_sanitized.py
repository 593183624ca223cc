"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (g++), driven
through every entry point on small ragged pictures: full, bounded, seeded and sub-pel
searches, listed CTU subsets, multi-threaded runs, intra prediction at the edges,
interpolation far outside the picture and depth bounds at odd ratios."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call([
        "g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
        os.path.join(ROOT, "oracle", "oracle.cpp"),
        os.path.join(ROOT, "tests", "cpp", "oracle_san_main.cpp"), "-o", exe])
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:] + res.stdout[-2000:]
    assert "all checks passed" in res.stdout
