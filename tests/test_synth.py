"""The seeded generators (CPU): the fragment image's single scatter writes
the same bytes as placing every copy in order; the tuning sample is never the
benchmark image; the batched images follow their specs."""
from dataclasses import replace

import torch

import synth


def test_fragment_image_equals_copies_in_order():
    # small image, many large copies: most of them overlap others
    cfg = synth.FragmentConfig("overlaps", 3, 20, 200, 3000, 1 << 16, 300, 0.7)
    files = synth.fragment_files(cfg)
    places = synth.fragment_placements(cfg, [f.numel() for f in files])
    spans = sorted((o, o + files[f].numel()) for o, f in places)
    assert sum(1 for a, b in zip(spans, spans[1:]) if b[0] < a[1]) > 50
    img = synth.fragment_image(cfg, files)
    ref = synth.fragment_image(replace(cfg, n_embedded=0), files)   # the random bytes alone
    for o, f in places:
        ref[o: o + files[f].numel()] = files[f]
    assert torch.equal(img, ref)


def test_tuning_sample_is_not_the_image():
    cfg = synth.scaled(synth.CONFIGS["mid"], n_master_sectors=4096, n_disk_sectors=4096, n_files=8)
    ms = synth.master_set(cfg)
    img = synth.disk_image(cfg, ms).data
    smp = synth.tuning_sample(cfg, ms, max_sectors=1024)
    assert smp.numel() == 1024 * 512
    assert not torch.equal(smp, img[: smp.numel()])


def test_batch_images_follow_specs():
    cfg = synth.scaled(synth.CONFIGS["mid"], n_master_sectors=4096, n_disk_sectors=1, n_files=8)
    ms = synth.master_set(cfg)
    specs = synth.batch_image_specs(seed=cfg.seed, n_images=3, max_bytes=1 << 21)
    imgs = synth.batch_images(cfg, ms, n_images=3)
    assert [t.numel() // 512 for t in imgs] == [n for n, _ in synth.batch_image_specs(seed=cfg.seed, n_images=3)]
    assert len(specs) == 3
