"""A small reader of the TIFF files the library writes, for the tests: parses
the header (classic or BigTIFF, little-endian), follows the IFD chain and
reassembles each tiled 8-bit RGBA image.  Independent of the writer."""
import struct

import numpy as np

TYPES = {3: ("H", 2), 4: ("I", 4), 16: ("Q", 8)}


def read(path):
    data = open(path, "rb").read()
    assert data[:2] == b"II", "little-endian only"
    magic = struct.unpack_from("<H", data, 2)[0]
    big = magic == 43
    assert magic in (42, 43)
    if big:
        assert struct.unpack_from("<HH", data, 4) == (8, 0)
        off = struct.unpack_from("<Q", data, 8)[0]
    else:
        off = struct.unpack_from("<I", data, 4)[0]
    levels = []
    while off:
        if big:
            n = struct.unpack_from("<Q", data, off)[0]
            p, esz = off + 8, 20
        else:
            n = struct.unpack_from("<H", data, off)[0]
            p, esz = off + 2, 12
        tags = {}
        prev = -1
        for i in range(n):
            e = p + i * esz
            if big:
                tag, typ, cnt = struct.unpack_from("<HHQ", data, e)
                vf, vsize = e + 12, 8
            else:
                tag, typ, cnt = struct.unpack_from("<HHI", data, e)
                vf, vsize = e + 8, 4
            assert tag > prev, "tags must be sorted"
            prev = tag
            fmt, sz = TYPES[typ]
            loc = vf if cnt * sz <= vsize else struct.unpack_from("<Q" if big else "<I", data, vf)[0]
            tags[tag] = list(struct.unpack_from("<" + fmt * cnt, data, loc))
        nxt = struct.unpack_from("<Q" if big else "<I", data, p + n * esz)[0]
        w, h = tags[256][0], tags[257][0]
        tw, th = tags[322][0], tags[323][0]
        img = np.zeros((h, w, 4), np.uint8)
        tx = (w + tw - 1) // tw
        for k, (o, c) in enumerate(zip(tags[324], tags[325])):
            assert c == tw * th * 4
            tile = np.frombuffer(data, np.uint8, c, o).reshape(th, tw, 4)
            j, i = divmod(k, tx)
            y0, x0 = j * th, i * tw
            img[y0:y0 + th, x0:x0 + tw] = tile[:min(th, h - y0), :min(tw, w - x0)]
        levels.append({"tags": tags, "image": img})
        off = nxt
    return {"bigtiff": big, "levels": levels}
