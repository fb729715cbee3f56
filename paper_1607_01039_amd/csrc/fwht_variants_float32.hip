// Tile-kernel variants for float32 entries (see wht_tile.hpp).
// Name: C<TB> = contiguous pass over tiles of 2^TB entries; S<TB>c<CB> =
// strided pass over tiles of 2^(TB-CB) rows x 2^CB contiguous columns, so it
// transforms up to TB-CB index bits per pass.
#include "fwht_internal.hpp"
#include "wht_contig16.hpp"
#include "wht_tile.hpp"

namespace fwht {

std::vector<Variant> variants_f32()
{
    using S = float;
    return {
        Variant{"C12", 12, 6, 256, true, &launch_tile<12, 6, 256, true, S, false>},
        Variant{"C13", 13, 6, 512, true, &launch_tile<13, 6, 512, true, S, false>},
        Variant{"C14", 14, 6, 512, true, &launch_tile<14, 6, 512, true, S, false>},
        Variant{"C15", 15, 6, 1024, true, &launch_tile<15, 6, 1024, true, S, false>},
        Variant{"C15p", 15, 6, 512, true, &launch_contig15p<S>, true},
        Variant{"C16", 16, 6, 1024, true, &launch_contig16<S>, true},
        // 2^16-entry strided tiles (two-round transposes), full height only
        Variant{"S16c7", 16, 7, 1024, false, &launch_pinned16<S, 7, 0>, true},
        Variant{"S16c8", 16, 8, 1024, false, &launch_pinned16<S, 8, 0>, true},
        Variant{"S16c9", 16, 9, 1024, false, &launch_pinned16<S, 9, 0>, true},
        // 2^15-entry strided tiles held by 512 threads (two workgroups per CU), full height only
        Variant{"S15c7p", 15, 7, 512, false, &launch_strided15p<S, 7>, true},
        Variant{"S15c8p", 15, 8, 512, false, &launch_strided15p<S, 8>, true},
        Variant{"S8c5", 8, 5, 64, false, &launch_tile<8, 5, 64, false, S, false>},
        Variant{"S9c5", 9, 5, 64, false, &launch_tile<9, 5, 64, false, S, false>},
        Variant{"S10c5", 10, 5, 64, false, &launch_tile<10, 5, 64, false, S, false>},
        Variant{"S11c5", 11, 5, 128, false, &launch_tile<11, 5, 128, false, S, false>},
        Variant{"S12c5", 12, 5, 256, false, &launch_tile<12, 5, 256, false, S, false>},
        Variant{"S13c5", 13, 5, 512, false, &launch_tile<13, 5, 512, false, S, false>},
        Variant{"S14c5", 14, 5, 512, false, &launch_tile<14, 5, 512, false, S, false>},
        Variant{"S8c6", 8, 6, 64, false, &launch_tile<8, 6, 64, false, S, false>},
        Variant{"S9c6", 9, 6, 64, false, &launch_tile<9, 6, 64, false, S, false>},
        Variant{"S10c6", 10, 6, 64, false, &launch_tile<10, 6, 64, false, S, false>},
        Variant{"S11c6", 11, 6, 128, false, &launch_tile<11, 6, 128, false, S, false>},
        Variant{"S12c6", 12, 6, 256, false, &launch_tile<12, 6, 256, false, S, false>},
        Variant{"S13c6", 13, 6, 512, false, &launch_tile<13, 6, 512, false, S, false>},
        Variant{"S14c6", 14, 6, 512, false, &launch_tile<14, 6, 512, false, S, false>},
        Variant{"S15c6", 15, 6, 1024, false, &launch_tile<15, 6, 1024, false, S, false>},
        Variant{"S8c7", 8, 7, 64, false, &launch_tile<8, 7, 64, false, S, false>},
        Variant{"S9c7", 9, 7, 64, false, &launch_tile<9, 7, 64, false, S, false>},
        Variant{"S10c7", 10, 7, 64, false, &launch_tile<10, 7, 64, false, S, false>},
        Variant{"S11c7", 11, 7, 128, false, &launch_tile<11, 7, 128, false, S, false>},
        Variant{"S12c7", 12, 7, 256, false, &launch_tile<12, 7, 256, false, S, false>},
        Variant{"S13c7", 13, 7, 512, false, &launch_tile<13, 7, 512, false, S, false>},
        Variant{"S14c7", 14, 7, 512, false, &launch_tile<14, 7, 512, false, S, false>},
        Variant{"S15c7", 15, 7, 1024, false, &launch_tile<15, 7, 1024, false, S, false>},
        Variant{"S9c8", 9, 8, 64, false, &launch_tile<9, 8, 64, false, S, false>},
        Variant{"S10c8", 10, 8, 64, false, &launch_tile<10, 8, 64, false, S, false>},
        Variant{"S11c8", 11, 8, 128, false, &launch_tile<11, 8, 128, false, S, false>},
        Variant{"S12c8", 12, 8, 256, false, &launch_tile<12, 8, 256, false, S, false>},
        Variant{"S13c8", 13, 8, 512, false, &launch_tile<13, 8, 512, false, S, false>},
        Variant{"S14c8", 14, 8, 512, false, &launch_tile<14, 8, 512, false, S, false>},
        Variant{"S15c8", 15, 8, 1024, false, &launch_tile<15, 8, 1024, false, S, false>},
        // twins with non-temporal loads and stores (the autotuner picks per size)
        Variant{"C15pn", 15, 6, 512, true, &launch_contig15p<S, NT_LOAD | NT_STORE>, true},
        Variant{"C16n", 16, 6, 1024, true, &launch_contig16<S, NT_LOAD | NT_STORE>, true},
        Variant{"S16c7n", 16, 7, 1024, false, &launch_pinned16<S, 7, NT_LOAD | NT_STORE>, true},
        Variant{"S16c8n", 16, 8, 1024, false, &launch_pinned16<S, 8, NT_LOAD | NT_STORE>, true},
        Variant{"S16c9n", 16, 9, 1024, false, &launch_pinned16<S, 9, NT_LOAD | NT_STORE>, true},
        Variant{"S15c7pn", 15, 7, 512, false, &launch_strided15p<S, 7, NT_LOAD | NT_STORE>, true},
        Variant{"S15c8pn", 15, 8, 512, false, &launch_strided15p<S, 8, NT_LOAD | NT_STORE>, true},
        Variant{"S13c5n", 13, 5, 512, false, &launch_tile<13, 5, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c5n", 14, 5, 512, false, &launch_tile<14, 5, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c6n", 13, 6, 512, false, &launch_tile<13, 6, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c6n", 14, 6, 512, false, &launch_tile<14, 6, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S15c6n", 15, 6, 1024, false, &launch_tile<15, 6, 1024, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c7n", 13, 7, 512, false, &launch_tile<13, 7, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c7n", 14, 7, 512, false, &launch_tile<14, 7, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S15c7n", 15, 7, 1024, false, &launch_tile<15, 7, 1024, false, S, NT_LOAD | NT_STORE>},
        Variant{"S13c8n", 13, 8, 512, false, &launch_tile<13, 8, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S14c8n", 14, 8, 512, false, &launch_tile<14, 8, 512, false, S, NT_LOAD | NT_STORE>},
        Variant{"S15c8n", 15, 8, 1024, false, &launch_tile<15, 8, 1024, false, S, NT_LOAD | NT_STORE>},
    };
}

}  // namespace fwht
