"""Host logic of bench.py (no GPU): the kernel-source hash that decides
whether the committed counter figures apply, the records read from them,
and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, kernels, device):
    d = tmp_path / 'paper_2411_11229_amd' / 'csrc'
    d.mkdir(parents=True)
    (d / 'hweno_kernels.hip').write_text(kernels)
    (d / 'hweno_device.h').write_text(device)
    return str(tmp_path)


def test_kernel_hash_ignores_comments_and_blank_space(tmp_path, monkeypatch):
    code = 'int f(int x) {\n  return x + 1;\n}\n'
    a = _tree(tmp_path / 'a', code, 'double g;\n')
    b = _tree(tmp_path / 'b', '// a comment\n' + code.replace('x + 1', 'x  +  1 /* one */'),
              '/* header\n   text */\ndouble g;  // trailing\n')
    c = _tree(tmp_path / 'c', code.replace('x + 1', 'x + 2'), 'double g;\n')
    hashes = []
    for root in (a, b, c):
        monkeypatch.setattr(bench, 'ROOT', root)
        hashes.append(bench.kernel_hash())
    assert hashes[0] == hashes[1]          # comments and spacing only
    assert hashes[0] != hashes[2]          # a change of code


def test_profile_records_follow_the_hash(tmp_path, monkeypatch):
    root = _tree(tmp_path, 'int k;\n', 'int d;\n')
    monkeypatch.setattr(bench, 'ROOT', root)
    prof = tmp_path / 'traffic.json'
    monkeypatch.setattr(bench, 'PROFILE_JSON', str(prof))
    assert bench.traffic_record() is None            # no record committed
    rec = dict(kernel_source_sha256=bench.kernel_hash(), traffic_bytes_per_launch=1.5e9,
               valu=dict(instructions_per_launch=1e8),
               f32=dict(traffic_bytes_per_launch=7e8, valu=dict(instructions_per_launch=9e7)))
    prof.write_text(json.dumps(rec))
    assert bench.traffic_record() == 1.5e9
    assert bench.traffic_record('f32') == 7e8
    assert bench.valu_record()['instructions_per_launch'] == 1e8
    assert bench.valu_record('f32')['instructions_per_launch'] == 9e7
    # taken on other sources: no figures
    rec['kernel_source_sha256'] = '0' * 64
    prof.write_text(json.dumps(rec))
    assert bench.traffic_record() is None and bench.valu_record('f32') is None


def test_committed_traffic_record_matches_the_sources():
    """The committed counter summary was taken on the kernels as they are."""
    rec = json.load(open(bench.PROFILE_JSON))
    assert rec['kernel_source_sha256'] == bench.kernel_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert 'one GPU' in r.stderr
