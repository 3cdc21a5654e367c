"""The fused assembly's incidence schedule (csrc/schedule.h, host code) on the
CPU: a small C++ driver built with AddressSanitizer and
UndefinedBehaviorSanitizer schedules every row of a few meshes, and the
invariant the assembly kernel's unserialized adds rely on is checked here:
every incidence of a row appears once, in steps of four whose elements share
no vertex but the row's."""
import os
import subprocess

import numpy as np
import pytest

import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1103_0066_amd", "csrc")

_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "schedule.h"
int main(int argc, char **argv)
{
    FILE *f = std::fopen(argv[1], "rb");
    int64_t hdr[3];                                   // n_vertices, n_elements, nv
    if (!f || std::fread(hdr, 8, 3, f) != 3) return 2;
    const int64_t Nv = hdr[0], E = hdr[1];
    const int nv = int(hdr[2]);
    std::vector<int32_t> conn(size_t(E) * nv);
    if (std::fread(conn.data(), 4, conn.size(), f) != conn.size()) return 3;
    std::fclose(f);
    std::vector<int32_t> ptr(size_t(Nv) + 1, 0), inc(conn.size());
    for (int32_t v : conn) ++ptr[size_t(v) + 1];
    for (int64_t v = 0; v < Nv; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
    for (size_t i = 0; i < conn.size(); ++i) inc[cur[conn[i]]++] = int32_t(i);
    std::vector<int32_t> sptr(size_t(Nv) + 1, 0), sinc;
    for (int64_t v = 0; v < Nv; ++v) {
        fei::schedule_row(int32_t(v), inc.data() + ptr[v], ptr[v + 1] - ptr[v], conn, nv, 4, sinc);
        sptr[v + 1] = int32_t(sinc.size());
    }
    f = std::fopen(argv[2], "wb");
    std::fwrite(sptr.data(), 4, sptr.size(), f);
    std::fwrite(sinc.data(), 4, sinc.size(), f);
    std::fclose(f);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("schedule")
    src = d / "drv.cpp"
    src.write_text(_DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", CSRC,
                    str(src), "-o", str(exe)], check=True)
    return d, exe


def _schedule(driver, conn, n_vertices):
    d, exe = driver
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    inp, out = d / "conn.bin", d / "sched.bin"
    with open(inp, "wb") as f:
        np.array([n_vertices, conn.shape[0], conn.shape[1]], np.int64).tofile(f)
        conn.tofile(f)
    r = subprocess.run([str(exe), str(inp), str(out)], capture_output=True, text=True,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"), timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    raw = np.fromfile(out, dtype=np.int32)
    return raw[:n_vertices + 1], raw[n_vertices + 1:]


@pytest.mark.parametrize("case", ["square", "kuhn", "fan", "degenerate"])
def test_schedule_steps_share_no_vertex_but_the_row(driver, case):
    if case == "square":
        m = meshgen.square_mesh(9, 0.2, 121, np.float32)
    elif case == "kuhn":
        m = meshgen.elast3d(10).mesh
    elif case == "fan":
        m = meshgen.fan_mesh(150, 122)
    else:   # elements listing a vertex twice or four times: their incidences of that
        # vertex never share a step
        base = meshgen.cube_mesh(2, 2, 2, 0.1, 123)
        conn = np.vstack([base.conn, [[0, 0, 1, 2], [5, 5, 5, 5], [5, 5, 7, 8]]]).astype(np.int32)
        m = meshgen.Mesh(base.coords, conn)
    ptr, inc = _schedule(driver, m.conn, m.n_vertices)
    nv = m.conn.shape[1]
    assert ptr[0] == 0 and ptr[-1] == len(inc) and np.all(np.diff(ptr) % 4 == 0)
    steps24 = tight = 0
    for v in range(m.n_vertices):
        ent = inc[ptr[v]:ptr[v + 1]]
        want = sorted(e * nv + a for e, row in enumerate(m.conn) for a, x in enumerate(row)
                      if x == v) if m.n_elements < 2000 else None
        if want is not None:
            assert sorted(ent[ent >= 0].tolist()) == want
        for st in ent.reshape(-1, 4):
            live = st[st >= 0]
            assert len(live) > 0                          # no empty step
            seen, elems = set(), set()
            for x in live:
                e, a = divmod(int(x), nv)
                assert m.conn[e, a] == v and e not in elems    # distinct elements
                elems.add(e)
                others = set(m.conn[e].tolist()) - {v}
                assert not (others & seen)
                seen |= others
        n = int((ent >= 0).sum())
        if n == 24:
            steps24 += 1
            tight += len(ent) == 24
    if case == "kuhn":
        assert steps24 > 0 and tight >= 0.99 * steps24
